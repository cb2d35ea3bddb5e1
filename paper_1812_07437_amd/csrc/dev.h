// Device-side helpers shared by the HIP kernels of libwlcov (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

namespace wlc {

constexpr int WAVE = 64;

// Everything a kernel needs about the tables and the plan, by value.
struct DevTables {
  const double *chi, *w_chi, *k, *m, *w_m, *W, *P, *u, *n_m, *b1, *b2;
  int n_z, n_chi, n_k, n_m_pts;
  double rho, k_max;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
  return v;
}

// Bracketing interval of kk on an increasing grid: kg[j] <= kk <= kg[j+1],
// t the fractional position in ln k.  Returns false outside the grid.
__device__ __forceinline__ bool bracket_lnk(const double *kg, int nk, double kk, int &j, double &t) {
  if (!(kk >= kg[0] && kk <= kg[nk - 1])) return false;
  int lo = 0, hi = nk - 1;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (kg[mid] <= kk) lo = mid; else hi = mid;
  }
  if (lo == nk - 1) lo = nk - 2;
  j = lo;
  t = (log(kk) - log(kg[lo])) / (log(kg[lo + 1]) - log(kg[lo]));
  return true;
}

// Round-to-nearest-even float -> bf16 bits (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Exponent e with x = f 2^e, f in [0.5, 1); 0 for x == 0.
__device__ __forceinline__ int exp2_of(double x) {
  int e = 0;
  if (x != 0.0) (void)frexp(x, &e);
  return e;
}

}  // namespace wlc
