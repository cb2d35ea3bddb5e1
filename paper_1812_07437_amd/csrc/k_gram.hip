// One-halo covariance as a Gram product G = A A^T over the flattened
// (chi, M) axis (eqs. CovPPNG, Ins5P, Ins6P with eq. General1h of Rizzato et
// al. 2019), computed on lower-triangle tiles only.
//
// Variants (MFMA on gfx950, wave64):
//   bf16     v_mfma_f32_32x32x16_bf16, FP32 accumulation;
//   bf16x3   the same instruction on split operands A = hi + lo:
//            hi hi^T + hi lo^T + lo hi^T (the lo lo^T term is dropped);
//   f32      v_mfma_f32_16x16x4_f32;
//   f64      v_mfma_f64_16x16x4_f64.
// Rows of A carry a power-of-two scale so that their largest entry lies in
// [0.5, 1); the caller undoes it exactly.
//
// Work decomposition: a workgroup owns one output tile (I >= J) of the lower
// triangle and one contiguous slice of K: 256 x 256 for the bf16 variants
// (8 wavefronts), 128 x 128 for f32 / f64 (4 wavefronts, 2 x 2).  The bf16
// operands are copied from global memory straight into LDS ahead of their
// products (two stages ahead for one product, one for the split product);
// the f32 / f64 ones are staged through registers, the next slice prefetched.
// Slices of K (split-K) are reduced in a fixed order by a second kernel, so
// results are deterministic.  A 256-row tile halves the operand bytes per
// flop against a 128-row one, which matters because tiles that share a panel
// rarely run in step closely enough to share it through L2.
//
// Tile schedule: the hardware hands workgroup b to XCD b mod 8, and each XCD
// has its own L2.  Work items follow a super-block order (8 x 8 tiles per
// block), so that the workgroups resident on one XCD at a time cover part of
// a super-block and stream the same operand panels through that XCD's L2.
// For the bf16 products the order is dealt to the XCDs in chunks of 32 items
// (one per resident workgroup), 8 chunks at a time, so that all XCDs work on
// neighbouring tiles together and the device-wide last-level cache serves
// each panel once to all of them (measured: the one-product Gram at large10
// 135 -> 115 ms against each XCD walking its own eighth of the order; chunks
// of 16 or 64 were no faster).  The f32 / f64 products keep contiguous runs
// per XCD.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "f64tile.h"
#include "kernels.h"

namespace wlc {

constexpr int TILE = 128;

// Lower-triangle tile t -> (I, J), I >= J (row-major over the triangle).
__device__ __forceinline__ void tri_tile(int64_t t, int &I, int &J) {
  int64_t i = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  I = (int)i;
  J = (int)(t - i * (i + 1) / 2);
}

constexpr int SB = 8;     // tiles per super-block side
constexpr int N_XCD = 8;  // XCDs per device; workgroup b runs on XCD b mod 8

// Lower-triangle tile t -> (I, J) in super-block order for nt tiles per side:
// strips of SB tile rows, each strip's super-blocks left to right, the tiles
// of a super-block row-major (the diagonal block holds its lower triangle).
// All strips but the last are full, and strip P starts at tile
// 32 P^2 + 4 P (= sum over p < P of 64 p + 36).
__device__ __forceinline__ void sb_tile(int64_t t, int nt, int &I, int &J) {
  const int64_t full = nt / SB;
  int64_t P = (int64_t)((sqrt(16.0 + 128.0 * (double)t) - 4.0) / 64.0);
  if (P > full) P = full;
  while (P < full && 32 * (P + 1) * (P + 1) + 4 * (P + 1) <= t) ++P;
  while (P > 0 && 32 * P * P + 4 * P > t) --P;
  const int64_t u = t - (32 * P * P + 4 * P);
  const int64_t rr = P < full ? SB : nt - SB * P;  // tile rows in this strip
  const int64_t off = rr * SB * P;                  // tiles left of the diagonal block
  if (u < off) {
    const int64_t Q = u / (rr * SB), v = u % (rr * SB);
    I = (int)(SB * P + v / SB);
    J = (int)(SB * Q + v % SB);
  } else {
    int i, j;
    tri_tile(u - off, i, j);
    I = (int)(SB * P + i);
    J = (int)(SB * P + j);
  }
}

// Workgroup -> (tile, split) for a grid padded to a multiple of N_XCD: XCD x
// takes work items [x per, (x + 1) per).  With split K, work items run over
// groups of GS consecutive tiles (super-block order), slice-outer within a
// group, so the workgroups resident on an XCD together multiply the same k
// slice of a few shared panels; shorter work items also keep them closer in
// step, so the panels are shared through L2.  Returns false for padding.
constexpr int GS = 32;

// Work item w of a product with n_work = tiles x n_split items -> (tile,
// split), in the order described above.
__device__ __forceinline__ void gram_item(int64_t w, int64_t n_work, int n_split, int nt, int &I, int &J,
                                          int &split) {
  const int64_t n_tiles = n_work / n_split;
  const int64_t grp = w / ((int64_t)GS * n_split), base = grp * GS;
  const int64_t gsz = n_tiles - base < GS ? n_tiles - base : GS;
  const int64_t u = w - grp * GS * n_split;
  split = (int)(u / gsz);
  sb_tile(base + u % gsz, nt, I, J);
}

// XC = 0: XCD x takes work items [x per, (x + 1) per) (per = grid / N_XCD).
// XC > 0: the item order is cut into groups of N_XCD XC items and XCD x
// takes items x XC .. x XC + XC - 1 of every group, so that the XCDs work on
// neighbouring items at the same time and fetch the same operand panels
// (which the device-wide last-level cache then serves once); the grid is a
// multiple of N_XCD XC.
template <int XC>
__device__ __forceinline__ bool gram_work(int64_t n_work, int n_split, int nt, int &I, int &J, int &split) {
  const int64_t x = blockIdx.x % N_XCD, j = blockIdx.x / N_XCD;
  int64_t w;
  if (XC == 0)
    w = x * ((int64_t)gridDim.x / N_XCD) + j;
  else
    w = (j / XC) * (N_XCD * XC) + x * XC + j % XC;
  if (w >= n_work) return false;
  gram_item(w, n_work, n_split, nt, I, J, split);
  return true;
}

constexpr int GRAM_XC = 32;  // bf16 items per XCD and group: its resident workgroups

// Slice 0 of a split-K product goes straight to the output, slice s > 0 to
// partial buffer s - 1; the reduction adds the partials in slice order.
template <typename T>
__device__ __forceinline__ T *gram_dst(T *out, T *partial, int split, int64_t part_stride) {
  return split == 0 ? out : partial + (int64_t)(split - 1) * part_stride;
}

// ===================================================================== bf16
// 256 x 256 output tile per workgroup of NW wavefronts on a 2 x (NW/2) grid:
// NW = 8 gives 128 x 64 per wavefront (4 x 2 blocks of
// v_mfma_f32_32x32x16_bf16, two wavefronts per SIMD).  K advances in stages
// of 32 through LDS stage buffers ([256 rows][32 bf16] = 64 B per row, operand
// and side).  Chunk c (16 B) of row r sits at slot c ^ (((r >> 1) ^ (r >> 3))
// & 3): the 16 consecutive rows that one MFMA operand read touches at a time
// then fall on 16 distinct 16-byte bank groups (and any 8 consecutive rows on
// 8), so operand reads are free of bank conflicts.
//
// Operands go straight from global memory into LDS (buffer loads with the
// LDS flag: lane l of a wavefront writes 16 bytes at the wavefront's LDS base
// + 16 l).  A is k-blocked (GRAM_KB = 32 columns per block), so one stage of
// a 256-row panel is a contiguous 16 KB block, and each 1 KB wavefront copy
// (16 rows) covers whole cache lines.  Lane l fills LDS slot l & 3 of row
// l >> 2 and fetches the chunk that the swizzle puts there (the swizzle is an
// XOR, its own inverse).  How many stages are in flight is the business of
// the tile bodies below (gram_bf16_tile1, gram_bf16_tile3).
constexpr int T2 = 256;
constexpr int BK2 = 32;
static_assert(BK2 == GRAM_KB, "a Gram stage is one k-block of A");
constexpr int GRAM_NW = 8;  // measured faster than 4 at both precisions

__device__ __forceinline__ int swz2(int r, int c) { return r * BK2 + ((c ^ (((r >> 1) ^ (r >> 3)) & 3)) << 3); }

// One stage of one operand: [side][T2 * BK2] (side 0 the rows of tile I,
// side 1 those of tile J).  Every stage buffer is a __shared__ array of its
// own, so the compiler can tell the buffer being filled from the ones being
// read and does not wait for a copy before reading another buffer.
typedef uint16_t GramStage[2][T2 * BK2];

// Wavefront w copies the 1 KB blocks idx = w PERW + q, q < PERW, of a stage's
// NOPS x 2 x 16 blocks (operand, side, 16-row group).  PERW divides 16, so a
// wavefront's blocks share operand and side, and its source is one panel.
template <int NOPS, int NW>
struct GramDma {
  static constexpr int PERW = NOPS * 2 * 16 / NW;
  static_assert(16 % PERW == 0, "a wavefront's blocks must share operand and side");
  uint32_t off[PERW];   // byte offset of this lane's chunk in the 16 KB panel stage
  const char *panel;    // the wavefront's panel at stage 0 (wavefront-uniform)
  int64_t stage_bytes;  // distance between consecutive k-blocks of A
  int blk0, op;
  __device__ __forceinline__ void init(const uint16_t *Ahi, const uint16_t *Alo, int64_t r_pad, int64_t row0,
                                       int64_t col0, int wave, int lane) {
    blk0 = wave * PERW;
    op = blk0 >> 5;
    const int side = (blk0 >> 4) & 1;
    panel = (const char *)((op == 0 ? Ahi : Alo) + (side == 0 ? row0 : col0) * BK2);
    stage_bytes = r_pad * BK2 * 2;
#pragma unroll
    for (int q = 0; q < PERW; ++q) {
      const int r = ((blk0 + q) & 15) * 16 + (lane >> 2);
      const int c = (lane & 3) ^ (((r >> 1) ^ (r >> 3)) & 3);
      off[q] = (uint32_t)(r * BK2 * 2 + 16 * c);
    }
  }
  // copy k-block kblk of the panel into the stage buffer of this wavefront's
  // operand; the copies are issued before anything that follows (the
  // scheduler would otherwise sink them below the products, next to the wait
  // for them)
  __device__ __forceinline__ void issue(int64_t kblk, GramStage &buf) const {
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void *)(panel + kblk * stage_bytes), 0, T2 * BK2 * 2, 0x00020000);
#pragma unroll
    for (int q = 0; q < PERW; ++q)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rsrc, (__attribute__((address_space(3))) void *)((char *)buf + ((blk0 + q) & 31) * 1024), 16, off[q], 0, 0,
          0);
    __builtin_amdgcn_sched_barrier(0);
  }
  __device__ __forceinline__ void issue(int64_t kblk, GramStage &hi, GramStage &lo) const {
    if (op == 0)
      issue(kblk, hi);
    else
      issue(kblk, lo);
  }
};

// Wait until at most N vector-memory operations of this wavefront are
// outstanding (s_waitcnt vmcnt(N), the other counters left alone).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt(0x0F70 | (N & 15) | ((N >> 4) << 14));
}

// Workgroup barrier without a memory fence: the callers wait for their own
// copies into LDS with wait_vmcnt first (a fence would wait for all of them,
// including the ones still meant to be in flight).  Every LDS read before it
// has been consumed by the products, so none is outstanding; lgkmcnt(0)
// states it.
__device__ __forceinline__ void stage_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// The products of one 32-k stage on a wavefront's 128 x WCOLS sub-tile:
// X3 false one product of the hi operands, true the split product.
template <bool X3, int NW>
struct GramAcc {
  static constexpr int WCOLS = 512 / NW;  // wavefront tile columns
  static constexpr int BJ = WCOLS / 32;   // 32-column blocks per wavefront
  f32x16 acc[4][BJ];
  int wr, wc, lane;
  __device__ __forceinline__ void init(int wave, int lane_) {
    lane = lane_;
    wr = (wave / (NW / 2)) * 128;
    wc = (wave % (NW / 2)) * WCOLS;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < BJ; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.0f;
  }
  __device__ __forceinline__ void stage(const GramStage &hi, const GramStage &lo) {
    constexpr int NOPS = X3 ? 2 : 1;
#pragma unroll
    for (int kk = 0; kk < BK2; kk += 16) {
      // lane holds 8 consecutive k of row (lane & 31), k offset 8 * (lane >> 5)
      const int cidx = (kk >> 3) + (lane >> 5);
      bf16x8 a[NOPS][4], b[NOPS][BJ];
#pragma unroll
      for (int op = 0; op < NOPS; ++op) {
        const GramStage &buf = op == 0 ? hi : lo;
#pragma unroll
        for (int blk = 0; blk < 4; ++blk)
          a[op][blk] = *(const bf16x8 *)(&buf[0][swz2(wr + blk * 32 + (lane & 31), cidx)]);
#pragma unroll
        for (int blk = 0; blk < BJ; ++blk)
          b[op][blk] = *(const bf16x8 *)(&buf[1][swz2(wc + blk * 32 + (lane & 31), cidx)]);
      }
      // products outermost, so consecutive MFMAs use different accumulators
#pragma unroll
      for (int p = 0; p < (X3 ? 3 : 1); ++p)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < BJ; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[p == 2 ? 1 : 0][i], b[p == 1 ? 1 : 0][j],
                                                                acc[i][j], 0, 0, 0);
    }
  }
  // 32x32 accumulator layout: value v of lane l is row 8 (v/4) + 4 (l/32) + v%4, column l % 32
  __device__ __forceinline__ void store(float *dst, int64_t row0, int64_t col0, int64_t ld) const {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < BJ; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t r = row0 + wr + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          const int64_t c = col0 + wc + j * 32 + (lane & 31);
          dst[r * ld + c] = acc[i][j][v];
        }
  }
};

// One work item with one product: tile (I, J), k slice split, through three
// stage buffers in a ring, each copy issued two stages ahead.  Before
// multiplying stage s a wavefront waits until its copy of stage s is in
// (only that of s + 1 may be outstanding), and after the barrier every
// wavefront's is, and the buffer of stage s - 1 is no longer read, so the
// copy of stage s + 2 goes there.  Two stages in flight per workgroup keep
// the operand stream busier than one (measured at 33280 rows, K = 131072:
// 114 -> 100 ms on operands with the sparsity of the one-halo factor).
template <int NW>
__device__ __forceinline__ void gram_bf16_tile1(const uint16_t *__restrict__ Ahi, int64_t k_pad, int64_t r_pad,
                                                int64_t k_split, int I, int J, int split, float *__restrict__ out,
                                                float *__restrict__ partial, int64_t ld, int64_t part_stride,
                                                GramStage &b0, GramStage &b1, GramStage &b2) {
  constexpr int PERW = GramDma<1, NW>::PERW;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t row0 = (int64_t)I * T2, col0 = (int64_t)J * T2;
  const int64_t kb = (int64_t)split * k_split;
  const int64_t ke = max(kb, min(k_pad, kb + k_split));  // an empty slice stores zeros
  GramAcc<false, NW> acc;
  acc.init(wave, lane);
  GramDma<1, NW> dma;
  dma.init(Ahi, Ahi, r_pad, row0, col0, wave, lane);
  const int64_t n_st = (ke - kb) / BK2, kb0 = kb / BK2;
  int64_t st = 0;
  if (n_st >= 5) {
    // the first two copies on the one path into the steady state, so that
    // the compiler's count of copies in flight at its top is exact (it would
    // otherwise wait for the second copy before reading the first)
    dma.issue(kb0, b0);
    dma.issue(kb0 + 1, b1);
  } else {
    if (n_st > 0) dma.issue(kb0, b0);
    if (n_st > 1) dma.issue(kb0 + 1, b1);
  }
  // steady state: every step issues the copy two stages ahead
  for (; st + 5 <= n_st; st += 3) {
    wait_vmcnt<PERW>();
    stage_barrier();
    dma.issue(kb0 + st + 2, b2);
    acc.stage(b0, b0);
    wait_vmcnt<PERW>();
    stage_barrier();
    dma.issue(kb0 + st + 3, b0);
    acc.stage(b1, b1);
    wait_vmcnt<PERW>();
    stage_barrier();
    dma.issue(kb0 + st + 4, b1);
    acc.stage(b2, b2);
  }
  // the last stages (fewer than five), waiting for every copy
  for (; st < n_st; st += 3) {
    wait_vmcnt<0>();
    stage_barrier();
    if (st + 2 < n_st) dma.issue(kb0 + st + 2, b2);
    acc.stage(b0, b0);
    if (st + 1 < n_st) {
      wait_vmcnt<0>();
      stage_barrier();
      if (st + 3 < n_st) dma.issue(kb0 + st + 3, b0);
      acc.stage(b1, b1);
    }
    if (st + 2 < n_st) {
      wait_vmcnt<0>();
      stage_barrier();
      if (st + 4 < n_st) dma.issue(kb0 + st + 4, b1);
      acc.stage(b2, b2);
    }
  }
  acc.store(gram_dst(out, partial, split, part_stride), row0, col0, ld);
}

// One work item with the split product: hi and lo of a stage in two buffers,
// two stages (b0, b1) and (b2, b3), stage s + 1 copied while stage s is
// multiplied.
template <int NW>
__device__ __forceinline__ void gram_bf16_tile3(const uint16_t *__restrict__ Ahi, const uint16_t *__restrict__ Alo,
                                                int64_t k_pad, int64_t r_pad, int64_t k_split, int I, int J,
                                                int split, float *__restrict__ out, float *__restrict__ partial,
                                                int64_t ld, int64_t part_stride, GramStage &b0, GramStage &b1,
                                                GramStage &b2, GramStage &b3) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t row0 = (int64_t)I * T2, col0 = (int64_t)J * T2;
  const int64_t kb = (int64_t)split * k_split;
  const int64_t ke = max(kb, min(k_pad, kb + k_split));  // an empty slice stores zeros
  GramAcc<true, NW> acc;
  acc.init(wave, lane);
  GramDma<2, NW> dma;
  dma.init(Ahi, Alo, r_pad, row0, col0, wave, lane);
  const int64_t n_st = (ke - kb) / BK2, kb0 = kb / BK2;
  if (n_st > 0) dma.issue(kb0, b0, b1);
  int64_t st = 0;
  for (; st + 1 < n_st; st += 2) {
    // this wavefront's copy of stage st is complete; after the barrier every
    // wavefront's is, and no wavefront still reads the buffers refilled next
    wait_vmcnt<0>();
    __syncthreads();
    dma.issue(kb0 + st + 1, b2, b3);
    acc.stage(b0, b1);
    wait_vmcnt<0>();
    __syncthreads();
    if (st + 2 < n_st) dma.issue(kb0 + st + 2, b0, b1);
    acc.stage(b2, b3);
  }
  if (st < n_st) {  // odd stage count: the last stage sits in (b0, b1)
    wait_vmcnt<0>();
    __syncthreads();
    acc.stage(b0, b1);
  }
  acc.store(gram_dst(out, partial, split, part_stride), row0, col0, ld);
}

// Products of the bf16 kernels: MODE 0 one bf16 product, MODE 1 the split
// product, MODE 2 per tile, the split product where the rows' largest
// one-halo shares F (per 256-row panel) give F_I F_J > lim and one product
// elsewhere (the split tiles are computed exactly as in MODE 1, the others
// as in MODE 0).
template <int MODE>
__device__ __forceinline__ bool tile_split(const double *__restrict__ panel_f, double lim, int I, int J) {
  if (MODE == 1) return true;
  if (MODE == 0) return false;
  return panel_f[I] * panel_f[J] > lim;
}

// With panel_ext, the k range of tile (I, J) ends after min(ext_I, ext_J)
// k-blocks (beyond it one of the two panels is zero), and the tile's slices
// split that range evenly, as the host splits the whole range without it, so
// that the work items of a product stay alike in length.
template <int MODE, int NW>
__device__ __forceinline__ void gram_bf16_item(const uint16_t *__restrict__ Ahi, const uint16_t *__restrict__ Alo,
                                               int64_t k_pad, int64_t r_pad, int64_t k_split, int n_split, int I,
                                               int J, int split, float *__restrict__ out, float *__restrict__ partial,
                                               int64_t ld, int64_t part_stride, const double *__restrict__ panel_f,
                                               double lim, const int32_t *__restrict__ panel_ext, GramStage &b0,
                                               GramStage &b1, GramStage &b2, GramStage &b3) {
  if (panel_ext) {
    k_pad = min(k_pad, (int64_t)max(min(panel_ext[I], panel_ext[J]), 0) * BK2);
    k_split = (k_pad / BK2 + n_split - 1) / n_split * BK2;
  }
  if (MODE != 0 && tile_split<MODE>(panel_f, lim, I, J))
    gram_bf16_tile3<NW>(Ahi, Alo, k_pad, r_pad, k_split, I, J, split, out, partial, ld, part_stride, b0, b1, b2, b3);
  else
    gram_bf16_tile1<NW>(Ahi, k_pad, r_pad, k_split, I, J, split, out, partial, ld, part_stride, b0, b1, b2);
}

template <int MODE, int NW>
__global__ __launch_bounds__(64 * NW) void k_gram_bf16(const uint16_t *__restrict__ Ahi, const uint16_t *__restrict__ Alo,
                                                  int64_t k_pad, int64_t r_pad, int64_t k_split, int n_split,
                                                  int nt, int64_t n_work, float *__restrict__ out,
                                                  float *__restrict__ partial, int64_t ld, int64_t part_stride,
                                                  const double *__restrict__ panel_f, double lim,
                                                  const int32_t *__restrict__ panel_ext) {
  __shared__ __attribute__((aligned(16))) GramStage b0;
  __shared__ __attribute__((aligned(16))) GramStage b1;
  __shared__ __attribute__((aligned(16))) GramStage b2;
  __shared__ __attribute__((aligned(16))) GramStage b3;  // split tiles only (unused, and not allocated, in MODE 0)
  int I, J, split;
  if (!gram_work<GRAM_XC>(n_work, n_split, nt, I, J, split)) return;
  gram_bf16_item<MODE, NW>(Ahi, Alo, k_pad, r_pad, k_split, n_split, I, J, split, out, partial, ld, part_stride,
                           panel_f, lim, panel_ext, b0, b1, b2, b3);
}

// ---------------------------------------------------------------- batched
// One persistent launch over the work items of several products (the Gram
// products of several requests of a server, each with its own operands,
// output, split-K choice and partial buffer).  Items are numbered product
// after product, each product's items in the order of gram_item, so that a
// product computes exactly what its own launch would (the same tiles, k
// slices and summation order).  The items are dealt to N_XCD queues as the
// direct launch deals them to XCDs (groups of N_XCD GRAM_XC items, GRAM_XC
// consecutive ones to each XCD); a workgroup claims items of its own XCD's
// queue (workgroup b runs on XCD b mod N_XCD) one at a time with an atomic
// counter, so the XCDs work on neighbouring items together, and moves on to
// the next queue when its own is drained.  Every workgroup leaves after
// finding all N_XCD queues drained, and items never wait for one another, so
// the grid drains whatever the residency.
constexpr int QSTRIDE = 16;  // counters 64 bytes apart

template <int MODE, int NW>
__global__ __launch_bounds__(64 * NW) void k_gram_bf16_batch(const GramJob *__restrict__ jobs, int n_jobs,
                                                        int64_t total, uint32_t *__restrict__ counters) {
  __shared__ __attribute__((aligned(16))) GramStage b0;
  __shared__ __attribute__((aligned(16))) GramStage b1;
  __shared__ __attribute__((aligned(16))) GramStage b2;
  __shared__ __attribute__((aligned(16))) GramStage b3;  // split tiles only (unused, and not allocated, in MODE 0)
  __shared__ int64_t s_item;
  const int x0 = blockIdx.x % N_XCD;
  int q = 0;
  constexpr int64_t GQ = (int64_t)N_XCD * GRAM_XC;
  const int64_t full = total / GQ, rest = total % GQ;
  while (q < N_XCD) {
    const int x = (x0 + q) % N_XCD;
    // queue x: items x GRAM_XC + g GQ + c, c < GRAM_XC, of every group g
    const int64_t tail = rest - (int64_t)x * GRAM_XC;
    const int64_t len = full * GRAM_XC + (tail < 0 ? 0 : (tail > GRAM_XC ? GRAM_XC : tail));
    __syncthreads();  // the previous item's LDS reads and s_item are done
    if (threadIdx.x == 0) {
      const int64_t c = (int64_t)atomicAdd(&counters[QSTRIDE * x], 1u);
      s_item = c < len ? (c / GRAM_XC) * GQ + (int64_t)x * GRAM_XC + c % GRAM_XC : -1;
    }
    __syncthreads();
    const int64_t g = s_item;
    if (g < 0) {
      ++q;
      continue;
    }
    int a = 0, b = n_jobs - 1;  // the job whose items hold g: largest item0 <= g
    while (a < b) {
      const int m = (a + b + 1) / 2;
      if (jobs[m].item0 <= g) a = m; else b = m - 1;
    }
    const GramJob &jb = jobs[a];
    int I, J, split;
    gram_item(g - jb.item0, jb.n_work, jb.n_split, jb.nt, I, J, split);
    gram_bf16_item<MODE, NW>((const uint16_t *)jb.A0, (const uint16_t *)jb.A1, jb.k_pad, jb.r_pad, jb.k_split,
                             jb.n_split, I, J, split, (float *)jb.out, (float *)jb.partial, jb.ld, jb.part_stride,
                             jb.panel_f, jb.split_lim, jb.panel_ext, b0, b1, b2, b3);
  }
}

__global__ void k_zero_u32(uint32_t *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// ===================================================================== f32 / f64
// v_mfma_f{32,64}_16x16x4: lane l holds element (row l % 16, k l / 16) of each
// operand; accumulator value v of lane l is column l % 16 and row 4 (l/16) + v
// for f32, row l/16 + 4 v for f64.  LDS rows are padded by one element.
template <typename T>
__device__ __forceinline__ void mfma16x16x4(T a, T b, typename std::conditional<sizeof(T) == 8, f64x4, f32x4>::type &c);

template <>
__device__ __forceinline__ void mfma16x16x4<double>(double a, double b, f64x4 &c) {
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ void mfma16x16x4<float>(float a, float b, f32x4 &c) {
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// With panel_ext (per 256-row panel the 32-column k-blocks where its rows can
// be nonzero), tile (I, J) sums only the k-blocks where both of its 256-row
// panels (I / 2 and J / 2) can be nonzero, split evenly over its slices; an
// empty slice stores zeros.  Items are dealt to the XCDs in chunks
// (gram_work<GRAM_XC>), which keeps the XCDs' shares of unequal items alike.
template <typename T>
__global__ __launch_bounds__(256) void k_gram_x4(const T *__restrict__ A, int64_t k_pad, int64_t lda, int64_t k_split,
                                                 int n_split, int nt, int64_t n_work, T *__restrict__ out,
                                                 T *__restrict__ partial, int64_t ld, int64_t part_stride,
                                                 const int32_t *__restrict__ panel_ext) {
  using acc_t = typename std::conditional<sizeof(T) == 8, f64x4, f32x4>::type;
  constexpr int BK = 128 / sizeof(T);  // 128 bytes of k per row
  constexpr int LDR = BK + 1;          // padded row length
  constexpr int CH = 16 / sizeof(T);   // elements per 16-byte chunk
  constexpr int NCH = TILE * BK / CH;  // chunks per operand tile
  constexpr int PER = NCH / 256;       // chunks per thread
  __shared__ T lds[2][TILE * LDR];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  int I, J, split;
  if (!gram_work<GRAM_XC>(n_work, n_split, nt, I, J, split)) return;
  const int64_t row0 = (int64_t)I * TILE, col0 = (int64_t)J * TILE;
  if (panel_ext) {
    k_pad = min(k_pad, (int64_t)max(min(panel_ext[I >> 1], panel_ext[J >> 1]), 0) * GRAM_KB);
    k_split = (k_pad / BK + n_split - 1) / n_split * BK;
  }
  const int64_t kb = (int64_t)split * k_split;
  const int64_t ke = min(k_pad, kb + k_split);
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;

  acc_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[a][b][v] = 0;

  typedef T vec_t __attribute__((ext_vector_type(CH)));
  vec_t pre[2][PER];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int64_t r0 = side == 0 ? row0 : col0;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int ch = tid + 256 * q;
        const int r = ch / (BK / CH), c = ch % (BK / CH);
        pre[side][q] = *(const vec_t *)(A + (r0 + r) * lda + k0 + CH * c);
      }
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int side = 0; side < 2; ++side)
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int ch = tid + 256 * q;
        const int r = ch / (BK / CH), c = ch % (BK / CH);
#pragma unroll
        for (int e = 0; e < CH; ++e) lds[side][r * LDR + CH * c + e] = pre[side][q][e];
      }
  };

  if (kb < ke) gload(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
    __syncthreads();
    lstore();
    __syncthreads();
    if (k0 + BK < ke) gload(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kq = kk + (lane >> 4);
      T a[4], b[4];
#pragma unroll
      for (int blk = 0; blk < 4; ++blk) {
        a[blk] = lds[0][(wr + blk * 16 + (lane & 15)) * LDR + kq];
        b[blk] = lds[1][(wc + blk * 16 + (lane & 15)) * LDR + kq];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) mfma16x16x4<T>(a[i], b[j], acc[i][j]);
    }
  }
  T *dst = gram_dst(out, partial, split, part_stride);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // f32: row 4 (l/16) + v; f64: row l/16 + 4 v (both column l % 16)
        const int64_t r = row0 + wr + i * 16 + (sizeof(T) == 8 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v);
        const int64_t c = col0 + wc + j * 16 + (lane & 15);
        dst[r * ld + c] = acc[i][j][v];
      }
}

// Fixed-order reduction of split-K partial tiles into the output (slice 0,
// then the partials in slice order).  Workgroup (t, h) takes rows
// 16 h .. 16 h + 15 of the 128 x 128 lower-triangle tile t, a thread one
// column of every other row, so that the launch has eight workgroups per
// tile (with one per tile, at the Euclid-like shape in FP64, 210 workgroups
// took 0.50 ms for 210 MB of partials).
constexpr int RED_ROWS = 16;
template <typename T>
__global__ __launch_bounds__(256) void k_gram_reduce(const T *__restrict__ part, int n_split, int64_t part_stride,
                                                     T *__restrict__ out, int64_t ld) {
  int I, J;
  tri_tile(blockIdx.x, I, J);
  const int64_t row0 = (int64_t)I * TILE + blockIdx.y * RED_ROWS + (threadIdx.x >> 7);
  const int64_t col = (int64_t)J * TILE + (threadIdx.x & 127);
#pragma unroll
  for (int q = 0; q < RED_ROWS / 2; ++q) {
    const int64_t off = (row0 + 2 * q) * ld + col;
    T s = out[off];  // slice 0
    for (int p = 1; p < n_split; ++p) s += part[(p - 1) * part_stride + off];
    out[off] = s;
  }
}

// FP64 Gram on 128 x 256 tiles with the tile product of f64tile.h: tile
// (I, J) covers rows [128 I, 128 I + 128) and columns [256 J, 256 J + 256)
// with J <= I / 2, which covers every 128 x 128 tile of the lower triangle
// (the diagonal ones with some entries above it, which the mirror
// overwrites).  Tiles are numbered by pairs of tile rows: rows 2m and 2m + 1
// hold m + 1 tiles each, so pair m starts at tile m (m + 1).  The rows are a
// multiple of 256, so every tile lies inside them.
__device__ __forceinline__ void f64_gram_tile(int64_t t, int &I, int &J) {
  int64_t m = (int64_t)((sqrt(4.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((m + 1) * (m + 2) <= t) ++m;
  while (m * (m + 1) > t) --m;
  const int64_t u = t - m * (m + 1);
  I = (int)(2 * m + u / (m + 1));
  J = (int)(u % (m + 1));
}

// With panel_ext (per 256-row panel the 32-column k-blocks where its rows can
// be nonzero), tile (I, J) sums only the k-blocks where both of its panels
// (the 256-row panel I / 2 and panel J) can be nonzero, and its slices split
// that range evenly; an empty slice stores zeros.
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_gram_f64(
    const double *__restrict__ A, int64_t k_pad, int64_t lda, int64_t k_split, int n_split, int64_t n_work,
    double *__restrict__ out, double *__restrict__ partial, int64_t ld, int64_t part_stride,
    const int32_t *__restrict__ panel_ext) {
  // items dealt to the XCDs in chunks of GRAM_XC (one per resident
  // workgroup), as gram_work<GRAM_XC> deals them: with panel extents the
  // items of the later panels are longer, and contiguous runs per XCD left
  // the last XCD 17 % more work than the mean at large10 (5 % dealt)
  const int64_t x = blockIdx.x % N_XCD, j = blockIdx.x / N_XCD;
  const int64_t w = (j / GRAM_XC) * (N_XCD * GRAM_XC) + x * GRAM_XC + j % GRAM_XC;
  if (w >= n_work) return;
  const int split = (int)(w % n_split);
  int I, J;
  f64_gram_tile(w / n_split, I, J);
  const int64_t row0 = (int64_t)I * FT_R, col0 = (int64_t)J * FT_S;
  if (panel_ext) {
    k_pad = min(k_pad, (int64_t)max(min(panel_ext[I >> 1], panel_ext[J]), 0) * GRAM_KB);
    k_split = (k_pad / FT_K + n_split - 1) / n_split * FT_K;
  }
  const int64_t kb = (int64_t)split * k_split;
  const int64_t ke = max(kb, min(k_pad, kb + k_split));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave / 4) * 64, wc = (wave % 4) * 64;
  f64x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  f64_tile_product(A + row0 * lda, A + col0 * lda, lda, FT_R, FT_S, kb, (ke - kb) / FT_K, acc);
  double *dst = gram_dst(out, partial, split, part_stride);
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = row0 + wr + x * 16 + (lane >> 4) + 4 * v;
        const int64_t c = col0 + wc + y * 16 + (lane & 15);
        dst[r * ld + c] = acc[x][y][v];
      }
}

// Mirror of the lower triangle onto the upper one in 64 x 64 tiles (I >= J):
// tile (I, J) is read row by row, transposed through LDS and written as tile
// (J, I), so both sides stay coalesced.  On a diagonal tile only the entries
// above the diagonal are written, after the whole tile has been read.  The
// upper side goes out with non-temporal stores (0.8 ms faster at 33280 rows).
template <typename T>
__global__ __launch_bounds__(256) void k_gram_mirror(T *__restrict__ G, int64_t ld) {
  __shared__ T tile[64][65];
  int I, J;
  tri_tile(blockIdx.x, I, J);
  const int c = threadIdx.x & 63, rb = (threadIdx.x >> 6) * 16;
  const int64_t i0 = (int64_t)I * 64, j0 = (int64_t)J * 64;
#pragma unroll
  for (int q = 0; q < 16; ++q) tile[rb + q][c] = G[(i0 + rb + q) * ld + j0 + c];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int r = rb + q;  // upper entry (j0 + r, i0 + c) = lower entry (i0 + c, j0 + r)
    if (I != J || c > r) __builtin_nontemporal_store(tile[c][r], &G[(j0 + r) * ld + i0 + c]);
  }
}

void launch_gram_mirror(int f32, void *G, int64_t n, int64_t ld, hipStream_t s) {
  const int64_t nt = (n + 63) / 64;  // nt * 64 <= ld: rows and columns are padded to the Gram tile
  const unsigned tiles = (unsigned)(nt * (nt + 1) / 2);
  if (f32)
    hipLaunchKernelGGL(k_gram_mirror<float>, dim3(tiles), dim3(256), 0, s, (float *)G, ld);
  else
    hipLaunchKernelGGL(k_gram_mirror<double>, dim3(tiles), dim3(256), 0, s, (double *)G, ld);
}

// G in the order of the distinct rows from the product of the A-rows (GP,
// symmetric): G[e][f] = GP[pos[e]][pos[f]], in 64 x 64 tiles of G.  Within a
// configuration the rows of one lowest bin are consecutive in both orders,
// so a wavefront's 64 reads of one GP row fall in a few contiguous runs.
template <typename T>
__global__ __launch_bounds__(256) void k_gram_unpermute(const T *__restrict__ GP, const int32_t *__restrict__ pos,
                                                       int64_t n, int64_t ld, T *__restrict__ G) {
  __shared__ int32_t prow[64];
  const int64_t nt = (n + 63) / 64;
  const int64_t I = blockIdx.x / nt, J = blockIdx.x % nt;
  const int c = threadIdx.x & 63, rb = (threadIdx.x >> 6) * 16;
  if (threadIdx.x < 64) prow[threadIdx.x] = I * 64 + threadIdx.x < n ? pos[I * 64 + threadIdx.x] : 0;
  __syncthreads();
  const int64_t f = J * 64 + c;
  if (f >= n) return;
  const int64_t pf = pos[f];
#pragma unroll 4
  for (int q = 0; q < 16; ++q) {
    const int64_t e = I * 64 + rb + q;
    if (e < n) G[e * ld + f] = GP[(int64_t)prow[rb + q] * ld + pf];
  }
}

void launch_gram_unpermute(int f32, const void *GP, const int32_t *pos, int64_t n, int64_t ld, void *G,
                           hipStream_t s) {
  const int64_t nt = (n + 63) / 64;
  if (f32)
    hipLaunchKernelGGL(k_gram_unpermute<float>, dim3((unsigned)(nt * nt)), dim3(256), 0, s, (const float *)GP, pos,
                       n, ld, (float *)G);
  else
    hipLaunchKernelGGL(k_gram_unpermute<double>, dim3((unsigned)(nt * nt)), dim3(256), 0, s, (const double *)GP, pos,
                       n, ld, (double *)G);
}

// Slices of K per tile.  Every slice beyond the first costs a Gram-sized
// partial buffer, its reduction and, per work item, a ring start-up and a
// 256 KB tile store.  The bf16 kernels run one 512-thread workgroup per CU;
// measured on the 256 x 128 (chi, M) grid (K = 32768) from 10 to 8515 tiles
// and at K = 131072, small products want few, long items: at 55 tiles one
// product took 0.23 ms with four slices and 0.96 ms with 32; at 90-230 tiles
// three or four slices were best, at 465-1275 tiles two; from about 2000
// tiles one slice is as fast as two or faster (11.5 against 12.1 ms at 8515
// tiles and K = 32768, equal at K = 131072) and needs no partial buffer.  The
// split product liked the same counts or somewhat more (8 below 100 tiles),
// within 2 % of its best beyond.  All bf16 modes take the same count, so a
// per-tile product (WLC_BF16_AUTO) sums each tile exactly as the one-product
// or the split-product mode would.  Each slice keeps at least 64 k-blocks.
// The FP32 and FP64 kernels aim at enough workgroups to cover the chip
// several times, with at least 4 K-steps per slice.
static int pick_split(int64_t n_tiles, int64_t k_pad, int bk, bool bf16) {
  const int64_t kb = k_pad / bk;
  int64_t s;
  if (bf16) {
    s = n_tiles >= 2048 ? 1 : std::clamp<int64_t>((600 + n_tiles - 1) / n_tiles, 2, 4);
    s = std::min<int64_t>(s, std::max<int64_t>(1, kb / 64));
  } else {
    const int64_t target = 2048;  // workgroups to cover 256 CUs several times
    s = (target + n_tiles - 1) / n_tiles;
    if (s > kb / 4) s = kb / 4;  // keep at least 4 K-steps per slice
    if (s < 1) s = 1;
    if (s > 32) s = 32;
  }
  return (int)s;
}

static bool is_bf16(int prec) { return prec == WLC_BF16 || prec == WLC_BF16X3 || prec == WLC_BF16_AUTO; }
static int bf16_mode(int prec) { return prec == WLC_BF16 ? 0 : (prec == WLC_BF16X3 ? 1 : 2); }
static int gram_tile(int prec) { return is_bf16(prec) ? T2 : TILE; }
static int gram_bk(int prec) { return prec == WLC_FP64 ? 16 : (prec == WLC_FP32 ? 32 : BK2); }
// the FP64 tile product needs even row pitch (16-byte chunks) and a 256-row
// panel within one buffer descriptor's 31-bit range
static bool f64_tiles(int prec, const GramShape &g) {
  return prec == WLC_FP64 && g.lda % 2 == 0 && (int64_t)FT_S * g.lda * 8 < ((int64_t)1 << 31) && g.r_pad % FT_S == 0;
}
bool gram_f64_tiles(const GramShape &g) { return f64_tiles(WLC_FP64, g); }
static int64_t gram_tile_count(int prec, const GramShape &g) {
  if (f64_tiles(prec, g)) {
    const int64_t pairs = g.r_pad / FT_S;
    return pairs * (pairs + 1);
  }
  const int64_t nt = g.r_pad / gram_tile(prec);
  return nt * (nt + 1) / 2;
}

size_t gram_partial_bytes(int prec, const GramShape &g) {
  const int s = pick_split(gram_tile_count(prec, g), g.k_pad, gram_bk(prec), is_bf16(prec));
  if (s <= 1) return 0;
  const size_t el = prec == WLC_FP64 ? 8 : 4;
  return (size_t)(s - 1) * g.r_pad * g.ld_out * el;  // slice 0 goes to the output
}

// Tiles, split-K slices and work items of one product: a function of its
// shape and precision only, so a product is computed the same way alone and
// in a batch.
struct GramSplit {
  int64_t nt, tiles, ksplit, pstride, n_work;
  int ns;
};

static GramSplit gram_split(int prec, const GramShape &g) {
  GramSplit q;
  q.nt = g.r_pad / gram_tile(prec);
  q.tiles = gram_tile_count(prec, g);
  const int bk = gram_bk(prec);
  q.ns = pick_split(q.tiles, g.k_pad, bk, is_bf16(prec));
  q.ksplit = (g.k_pad / bk + q.ns - 1) / q.ns * bk;
  q.pstride = q.ns > 1 ? g.r_pad * g.ld_out : 0;
  q.n_work = q.tiles * q.ns;
  return q;
}

bool gram_batchable(int prec) { return is_bf16(prec); }

void gram_job(int prec, const GramShape &g, const void *A0, const void *A1, void *out, void *partial, GramJob &job,
              const double *panel_f, double split_lim, const int32_t *panel_ext) {
  const GramSplit q = gram_split(prec, g);
  job.panel_f = panel_f;
  job.panel_ext = panel_ext;
  job.split_lim = split_lim;
  job.A0 = A0;
  job.A1 = A1;
  job.out = out;
  job.partial = partial;
  job.r_pad = g.r_pad;
  job.k_pad = g.k_pad;
  job.k_split = q.ksplit;
  job.ld = g.ld_out;
  job.part_stride = q.pstride;
  job.n_work = q.n_work;
  job.item0 = 0;
  job.n_split = q.ns;
  job.nt = (int32_t)q.nt;
}

// Workgroups of the batched kernel that fit on the device at once (the grid
// of the persistent launch), a multiple of N_XCD.
template <int MODE>
static int batch_slots() {
  static int slots = 0;  // per process: every device here is the same part
  if (!slots) {
    int dev = 0, cus = 0, occ = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_gram_bf16_batch<MODE, GRAM_NW>, 64 * GRAM_NW, 0) !=
            hipSuccess || occ <= 0)
      occ = 1;
    slots = (cus * occ + N_XCD - 1) / N_XCD * N_XCD;
  }
  return slots;
}

int launch_gram_batch(int prec, const GramJob *jobs_dev, int n_jobs, int64_t total, uint32_t *counters,
                      hipStream_t s) {
  if (!gram_batchable(prec) || n_jobs < 1 || total < 1) return -1;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(GRAM_BATCH_COUNTERS), 0, s, counters, GRAM_BATCH_COUNTERS);
  const int mode = bf16_mode(prec);
  const int64_t slots = mode == 0 ? batch_slots<0>() : (mode == 1 ? batch_slots<1>() : batch_slots<2>());
  const unsigned grid = (unsigned)std::min<int64_t>(slots, (total + N_XCD - 1) / N_XCD * N_XCD);
  if (mode == 0)
    hipLaunchKernelGGL((k_gram_bf16_batch<0, GRAM_NW>), dim3(grid), dim3(64 * GRAM_NW), 0, s, jobs_dev, n_jobs, total,
                       counters);
  else if (mode == 1)
    hipLaunchKernelGGL((k_gram_bf16_batch<1, GRAM_NW>), dim3(grid), dim3(64 * GRAM_NW), 0, s, jobs_dev, n_jobs, total,
                       counters);
  else
    hipLaunchKernelGGL((k_gram_bf16_batch<2, GRAM_NW>), dim3(grid), dim3(64 * GRAM_NW), 0, s, jobs_dev, n_jobs, total,
                       counters);
  return 0;
}

void launch_gram_reduce(int prec, const GramShape &g, void *out, void *partial, hipStream_t s) {
  const GramSplit q = gram_split(prec, g);
  if (q.ns <= 1) return;
  // the reduction walks the lower triangle in 128 x 128 tiles, which the
  // 256 x 256 tiles cover exactly
  const int64_t nr = g.r_pad / TILE;
  const unsigned rt = (unsigned)(nr * (nr + 1) / 2);
  const dim3 grid(rt, TILE / RED_ROWS);
  if (prec == WLC_FP64)
    hipLaunchKernelGGL(k_gram_reduce<double>, grid, dim3(256), 0, s, (const double *)partial, q.ns, q.pstride,
                       (double *)out, g.ld_out);
  else
    hipLaunchKernelGGL(k_gram_reduce<float>, grid, dim3(256), 0, s, (const float *)partial, q.ns, q.pstride,
                       (float *)out, g.ld_out);
}

void launch_gram(int prec, const GramShape &g, const void *A0, const void *A1, void *out, void *partial,
                 hipStream_t s, const double *panel_f, double split_lim, const int32_t *panel_ext) {
  const GramSplit q = gram_split(prec, g);
  const int64_t nt = q.nt, tiles = q.tiles, ksplit = q.ksplit, pstride = q.pstride, n_work = q.n_work;
  const int ns = q.ns;
  const int64_t gq = (int64_t)N_XCD * GRAM_XC;  // whole item groups of the dealt schedules
  const dim3 grid((unsigned)((n_work + gq - 1) / gq * gq));
  const int nti = (int)nt;
  switch (prec) {
    case WLC_BF16:
      hipLaunchKernelGGL((k_gram_bf16<0, GRAM_NW>), grid, dim3(64 * GRAM_NW), 0, s, (const uint16_t *)A0,
                         (const uint16_t *)A1, g.k_pad, g.r_pad, ksplit, ns, nti, n_work, (float *)out, (float *)partial,
                         g.ld_out, pstride, panel_f, split_lim, panel_ext);
      break;
    case WLC_BF16X3:
      hipLaunchKernelGGL((k_gram_bf16<1, GRAM_NW>), grid, dim3(64 * GRAM_NW), 0, s, (const uint16_t *)A0,
                         (const uint16_t *)A1, g.k_pad, g.r_pad, ksplit, ns, nti, n_work, (float *)out, (float *)partial,
                         g.ld_out, pstride, panel_f, split_lim, panel_ext);
      break;
    case WLC_BF16_AUTO:
      hipLaunchKernelGGL((k_gram_bf16<2, GRAM_NW>), grid, dim3(64 * GRAM_NW), 0, s, (const uint16_t *)A0,
                         (const uint16_t *)A1, g.k_pad, g.r_pad, ksplit, ns, nti, n_work, (float *)out, (float *)partial,
                         g.ld_out, pstride, panel_f, split_lim, panel_ext);
      break;
    case WLC_FP32:
      hipLaunchKernelGGL(k_gram_x4<float>, grid, dim3(256), 0, s, (const float *)A0, g.k_pad, g.lda, ksplit, ns, nti,
                         n_work, (float *)out, (float *)partial, g.ld_out, pstride, panel_ext);
      break;
    default:
      if (f64_tiles(prec, g)) {
        hipLaunchKernelGGL(k_gram_f64, grid, dim3(512), 0, s, (const double *)A0, g.k_pad, g.lda, ksplit, ns, n_work,
                           (double *)out, (double *)partial, g.ld_out, pstride, panel_ext);
        break;
      }
      hipLaunchKernelGGL(k_gram_x4<double>, grid, dim3(256), 0, s, (const double *)A0, g.k_pad, g.lda, ksplit, ns, nti,
                         n_work, (double *)out, (double *)partial, g.ld_out, pstride, panel_ext);
      break;
  }
  (void)tiles;
  launch_gram_reduce(prec, g, out, partial, s);
}

}  // namespace wlc
