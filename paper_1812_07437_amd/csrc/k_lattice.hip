// Integer lattice counts of modes and triangles (Rizzato et al. 2019,
// Sec. 3.2.2 mode lattice and App. B, N_tri as the sum of the selection
// function Delta^(3)).
//
// Modes are integer vectors q != 0; bin b holds q with T_b <= |q|^2 < T_{b+1}.
// The triangle count of bins (b1, b2, b3) is the number of ordered pairs
// (q1, q2) with q1 in b1, q2 in b2 and q1 + q2 in b3.  For a fixed q1 the
// admissible q2 of one lattice row form at most two intervals for each
// annulus condition, so each row is counted by interval intersection with
// exact integer square roots.  The count for q1 is invariant under the 8
// symmetries of the square lattice (applied to q2 as well), so only q1 with
// 0 <= y <= x are visited, with multiplicity 8, 4 (on an axis or a diagonal).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace wlc {

// floor(sqrt(v)) for v >= 0, exact in 64-bit integers
__device__ __forceinline__ int64_t isqrt_floor(int64_t v) {
  if (v <= 0) return 0;
  int64_t r = (int64_t)sqrt((double)v);
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

// x with lo <= x^2 + yy < hi, as up to two disjoint intervals [a0,b0], [a1,b1]
// (empty when a > b).  Returns the number of intervals written.
__device__ __forceinline__ int row_intervals(int64_t lo, int64_t hi, int64_t yy, int64_t *a, int64_t *b) {
  const int64_t top = hi - 1 - yy;  // x^2 <= top
  if (top < 0) return 0;
  const int64_t xmax = isqrt_floor(top);
  const int64_t need = lo - yy;  // x^2 >= need
  int64_t xmin = 0;
  if (need > 0) {
    xmin = isqrt_floor(need - 1) + 1;  // smallest x >= 0 with x^2 >= need
  }
  if (xmin > xmax) return 0;
  if (xmin == 0) {
    a[0] = -xmax; b[0] = xmax;
    return 1;
  }
  a[0] = -xmax; b[0] = -xmin;
  a[1] = xmin; b[1] = xmax;
  return 2;
}

__device__ __forceinline__ int64_t overlap(int64_t a0, int64_t b0, int64_t a1, int64_t b1) {
  const int64_t lo = a0 > a1 ? a0 : a1, hi = b0 < b1 ? b0 : b1;
  return hi >= lo ? hi - lo + 1 : 0;
}

// Number of q2 in bin 2 with q1 + q2 in bin 3.
__device__ uint64_t count_for_q1(int64_t x1, int64_t y1, int64_t lo2, int64_t hi2, int64_t lo3, int64_t hi3) {
  const int64_t r2 = isqrt_floor(hi2 - 1);
  uint64_t c = 0;
  for (int64_t y2 = -r2; y2 <= r2; ++y2) {
    int64_t a2[2], b2[2], a3[2], b3[2];
    const int n2 = row_intervals(lo2, hi2, y2 * y2, a2, b2);
    if (!n2) continue;
    const int64_t ys = y1 + y2;
    const int n3 = row_intervals(lo3, hi3, ys * ys, a3, b3);
    for (int p = 0; p < n2; ++p)
      for (int q = 0; q < n3; ++q) c += (uint64_t)overlap(a2[p], b2[p], a3[q] - x1, b3[q] - x1);
  }
  return c;
}

// grid: (row y1 of q1, triangle); threads stride over x1 >= y1 of that row.
__global__ __launch_bounds__(256) void k_lattice_tris(const int64_t *__restrict__ thr, const int32_t *__restrict__ tri,
                                                      uint64_t *__restrict__ out) {
  __shared__ uint64_t part[256];
  const int t = blockIdx.y;
  const int64_t y1 = blockIdx.x;
  const int b1 = tri[3 * t], b2 = tri[3 * t + 1], b3 = tri[3 * t + 2];
  const int64_t lo1 = thr[b1], hi1 = thr[b1 + 1];
  const int64_t lo2 = thr[b2], hi2 = thr[b2 + 1], lo3 = thr[b3], hi3 = thr[b3 + 1];
  uint64_t c = 0;
  const int64_t yy = y1 * y1;
  if (2 * yy < hi1) {  // some x >= y1 may still lie below the outer radius
    const int64_t xmax = isqrt_floor(hi1 - 1 - yy);
    int64_t xmin = y1;
    if (lo1 - yy > 0) {
      const int64_t m = isqrt_floor(lo1 - yy - 1) + 1;
      if (m > xmin) xmin = m;
    }
    for (int64_t x1 = xmin + threadIdx.x; x1 <= xmax; x1 += blockDim.x) {
      const uint64_t mult = (y1 == 0 || x1 == y1) ? 4 : 8;
      c += mult * count_for_q1(x1, y1, lo2, hi2, lo3, hi3);
    }
  }
  part[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && part[0]) atomicAdd((unsigned long long *)&out[t], (unsigned long long)part[0]);
}

__global__ void k_zero_u64(uint64_t *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// modes per bin: one thread per (bin, row y)
__global__ void k_lattice_modes(const int64_t *__restrict__ thr, int n_ell, int64_t rmax, uint64_t *__restrict__ out) {
  const int b = blockIdx.y;
  const int64_t lo = thr[b], hi = thr[b + 1];
  uint64_t c = 0;
  for (int64_t y = -rmax + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; y <= rmax;
       y += (int64_t)gridDim.x * blockDim.x) {
    int64_t a[2], bb[2];
    const int n = row_intervals(lo, hi, y * y, a, bb);
    for (int p = 0; p < n; ++p) c += (uint64_t)(bb[p] - a[p] + 1);
  }
  if (c) atomicAdd((unsigned long long *)&out[b], (unsigned long long)c);
}

// Full launch helpers with the host-known radius bound.
void launch_lattice(const int64_t *thr_dev, int64_t thr_max, int n_ell, const int32_t *tri, int n_tri,
                    uint64_t *modes, uint64_t *tris, hipStream_t s) {
  const int64_t rmax = (int64_t)std::sqrt((double)thr_max) + 2;
  if (modes) {
    hipLaunchKernelGGL(k_zero_u64, dim3((n_ell + 255) / 256), dim3(256), 0, s, modes, n_ell);
    hipLaunchKernelGGL(k_lattice_modes, dim3(8, n_ell), dim3(256), 0, s, thr_dev, n_ell, rmax, modes);
  }
  if (tris && n_tri > 0) {
    hipLaunchKernelGGL(k_zero_u64, dim3((n_tri + 255) / 256), dim3(256), 0, s, tris, n_tri);
    hipLaunchKernelGGL(k_lattice_tris, dim3((unsigned)rmax, (unsigned)n_tri), dim3(256), 0, s, thr_dev, tri, tris);
  }
}

}  // namespace wlc
