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
// Work decomposition: a workgroup of 4 wavefronts owns one 128 x 128 output
// tile (I >= J) and one contiguous slice of K; wavefronts split the tile 2 x 2.
// Operands are staged through LDS with the next slice prefetched into
// registers.  Slices of K (split-K) are reduced in a fixed order by a second
// kernel, so results are deterministic.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace wlc {

constexpr int TILE = 128;

// Lower-triangle tile t -> (I, J), I >= J.
__device__ __forceinline__ void tri_tile(int64_t t, int &I, int &J) {
  int64_t i = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  I = (int)i;
  J = (int)(t - i * (i + 1) / 2);
}

// ===================================================================== bf16
// LDS tile: [128 rows][64 bf16] = 128 B per row, in 16-byte chunks; chunk c of
// row r is stored at slot c ^ (r & 7) so that the 8 rows read together by an
// MFMA operand load hit distinct banks.
constexpr int BK16 = 64;

template <bool X3>
__global__ __launch_bounds__(256) void k_gram_bf16(const uint16_t *__restrict__ Ahi, const uint16_t *__restrict__ Alo,
                                                  int64_t k_pad, int64_t k_split, int n_split, float *__restrict__ out,
                                                  int64_t ld, int64_t part_stride) {
  constexpr int NOPS = X3 ? 2 : 1;  // hi (and lo)
  __shared__ __attribute__((aligned(16))) uint16_t lds[NOPS][2][TILE * BK16];  // [op][I/J][...]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t tile = blockIdx.x / n_split;
  const int split = blockIdx.x % n_split;
  int I, J;
  tri_tile(tile, I, J);
  const int64_t row0 = (int64_t)I * TILE, col0 = (int64_t)J * TILE;
  const int64_t kb = (int64_t)split * k_split;
  const int64_t ke = min(k_pad, kb + k_split);
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;  // wave sub-tile origin

  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.0f;

  // global -> register prefetch: 1024 chunks of 16 B per operand tile,
  // 4 per thread; chunk q: row q >> 3, chunk q & 7.
  u32x4 pre[NOPS][2][4];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int op = 0; op < NOPS; ++op) {
      const uint16_t *src = op == 0 ? Ahi : Alo;
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int64_t r0 = side == 0 ? row0 : col0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int ch = tid + 256 * q;
          const int r = ch >> 3, c = ch & 7;
          pre[op][side][q] = *(const u32x4 *)(src + (r0 + r) * k_pad + k0 + 8 * c);
        }
      }
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int op = 0; op < NOPS; ++op)
#pragma unroll
      for (int side = 0; side < 2; ++side)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int ch = tid + 256 * q;
          const int r = ch >> 3, c = ch & 7;
          *(u32x4 *)(&lds[op][side][r * BK16 + ((c ^ (r & 7)) << 3)]) = pre[op][side][q];
        }
  };

  if (kb < ke) gload(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += BK16) {
    __syncthreads();
    lstore();
    __syncthreads();
    if (k0 + BK16 < ke) gload(k0 + BK16);
#pragma unroll
    for (int kk = 0; kk < BK16; kk += 16) {
      // lane holds 8 consecutive k of row (lane & 31), k offset 8 * (lane >> 5)
      const int cidx = (kk >> 3) + (lane >> 5);
      bf16x8 a[NOPS][2], b[NOPS][2];
#pragma unroll
      for (int op = 0; op < NOPS; ++op)
#pragma unroll
        for (int blk = 0; blk < 2; ++blk) {
          const int ra = wr + blk * 32 + (lane & 31);
          const int rb = wc + blk * 32 + (lane & 31);
          a[op][blk] = *(const bf16x8 *)(&lds[op][0][ra * BK16 + ((cidx ^ (ra & 7)) << 3)]);
          b[op][blk] = *(const bf16x8 *)(&lds[op][1][rb * BK16 + ((cidx ^ (rb & 7)) << 3)]);
        }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0][i], b[0][j], acc[i][j], 0, 0, 0);
          if constexpr (X3) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0][i], b[1][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1][i], b[0][j], acc[i][j], 0, 0, 0);
          }
        }
    }
  }
  // 32x32 accumulator layout: value v of lane l is row 8 (v/4) + 4 (l/32) + v%4, column l % 32
  float *dst = out + (int64_t)split * part_stride;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t r = row0 + wr + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int64_t c = col0 + wc + j * 32 + (lane & 31);
        dst[r * ld + c] = acc[i][j][v];
      }
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

template <typename T>
__global__ __launch_bounds__(256) void k_gram_x4(const T *__restrict__ A, int64_t k_pad, int64_t k_split, int n_split,
                                                 T *__restrict__ out, int64_t ld, int64_t part_stride) {
  using acc_t = typename std::conditional<sizeof(T) == 8, f64x4, f32x4>::type;
  constexpr int BK = 128 / sizeof(T);  // 128 bytes of k per row
  constexpr int LDR = BK + 1;          // padded row length
  constexpr int CH = 16 / sizeof(T);   // elements per 16-byte chunk
  constexpr int NCH = TILE * BK / CH;  // chunks per operand tile
  constexpr int PER = NCH / 256;       // chunks per thread
  __shared__ T lds[2][TILE * LDR];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t tile = blockIdx.x / n_split;
  const int split = blockIdx.x % n_split;
  int I, J;
  tri_tile(tile, I, J);
  const int64_t row0 = (int64_t)I * TILE, col0 = (int64_t)J * TILE;
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
        pre[side][q] = *(const vec_t *)(A + (r0 + r) * k_pad + k0 + CH * c);
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
  T *dst = out + (int64_t)split * part_stride;
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

// Fixed-order reduction of split-K partial tiles into the output.
template <typename T>
__global__ void k_gram_reduce(const T *__restrict__ part, int n_split, int64_t part_stride, T *__restrict__ out,
                              int64_t ld) {
  const int64_t tile = blockIdx.x;
  int I, J;
  tri_tile(tile, I, J);
  const int64_t row0 = (int64_t)I * TILE, col0 = (int64_t)J * TILE;
  for (int e = threadIdx.x; e < TILE * TILE; e += blockDim.x) {
    const int64_t off = (row0 + e / TILE) * ld + col0 + e % TILE;
    T s = part[off];
    for (int q = 1; q < n_split; ++q) s += part[q * part_stride + off];
    out[off] = s;
  }
}

static int pick_split(int64_t n_tiles, int64_t k_pad, int bk) {
  const int64_t target = 2048;  // workgroups to cover 256 CUs several times
  int64_t s = (target + n_tiles - 1) / n_tiles;
  const int64_t kb = k_pad / bk;
  if (s > kb / 4) s = kb / 4;  // keep at least 4 K-steps per slice
  if (s < 1) s = 1;
  if (s > 32) s = 32;
  return (int)s;
}

static int gram_bk(int prec) { return prec == WLC_FP64 ? 16 : (prec == WLC_FP32 ? 32 : BK16); }

size_t gram_partial_bytes(int prec, const GramShape &g) {
  const int64_t nt = g.r_pad / TILE;
  const int64_t tiles = nt * (nt + 1) / 2;
  const int s = pick_split(tiles, g.k_pad, gram_bk(prec));
  if (s <= 1) return 0;
  const size_t el = prec == WLC_FP64 ? 8 : 4;
  return (size_t)s * g.r_pad * g.ld_out * el;
}

void launch_gram(int prec, const GramShape &g, const void *A0, const void *A1, void *out, void *partial,
                 hipStream_t s) {
  const int64_t nt = g.r_pad / TILE;
  const int64_t tiles = nt * (nt + 1) / 2;
  const int bk = gram_bk(prec);
  const int ns = pick_split(tiles, g.k_pad, bk);
  int64_t ksplit = (g.k_pad / bk + ns - 1) / ns * bk;
  void *dst = ns > 1 ? partial : out;
  const int64_t pstride = ns > 1 ? g.r_pad * g.ld_out : 0;
  const dim3 grid((unsigned)(tiles * ns));
  switch (prec) {
    case WLC_BF16:
      hipLaunchKernelGGL(k_gram_bf16<false>, grid, dim3(256), 0, s, (const uint16_t *)A0, (const uint16_t *)A1, g.k_pad,
                         ksplit, ns, (float *)dst, g.ld_out, pstride);
      break;
    case WLC_BF16X3:
      hipLaunchKernelGGL(k_gram_bf16<true>, grid, dim3(256), 0, s, (const uint16_t *)A0, (const uint16_t *)A1, g.k_pad,
                         ksplit, ns, (float *)dst, g.ld_out, pstride);
      break;
    case WLC_FP32:
      hipLaunchKernelGGL(k_gram_x4<float>, grid, dim3(256), 0, s, (const float *)A0, g.k_pad, ksplit, ns, (float *)dst,
                         g.ld_out, pstride);
      break;
    default:
      hipLaunchKernelGGL(k_gram_x4<double>, grid, dim3(256), 0, s, (const double *)A0, g.k_pad, ksplit, ns,
                         (double *)dst, g.ld_out, pstride);
      break;
  }
  if (ns > 1) {
    if (prec == WLC_FP64)
      hipLaunchKernelGGL(k_gram_reduce<double>, dim3((unsigned)tiles), dim3(256), 0, s, (const double *)partial, ns,
                         pstride, (double *)out, g.ld_out);
    else
      hipLaunchKernelGGL(k_gram_reduce<float>, dim3((unsigned)tiles), dim3(256), 0, s, (const float *)partial, ns,
                         pstride, (float *)out, g.ld_out);
  }
}

}  // namespace wlc
