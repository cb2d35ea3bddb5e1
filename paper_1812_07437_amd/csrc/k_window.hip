// Variance of the long background mode in the survey disk, for the
// super-sample term resolved along the line of sight.
//
// Rizzato et al. (2019), arXiv 1812.07437: sigma_W^2(chi) is defined after
// eq. CovPP22 (Sec. 3.2.3); the disk is the thin-shell limit of the cylinder
// window of eq. Mask (App. B).  In polar coordinates,
//   sigma_W^2(chi) = (2 / pi) int eps^2 [J1(x) / x]^2 P(eps, chi) d ln eps,
//   x = eps chi Theta,
// with Theta the survey's angular radius, Omega = 2 pi (1 - cos Theta) (the
// relation given after eq. PSest, Sec. 3.2.2).  The integral runs over the k table by the trapezoid rule in ln eps
// on WINDOW_NODES uniformly spaced nodes, the two end nodes being the table's
// first and last k; P is read by the table interpolation of every other
// kernel (linear in ln P against ln k).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace wlc {

constexpr double PI_D = 3.14159265358979323846;

// Bessel function of the first kind of order one, x > 0 (Abramowitz &
// Stegun, ch. 9):
//   x < 2        its power series (9.1.10), terms falling at least 6-fold;
//   2 <= x < 25  Bessel's integral J1(x) = (1/pi) int_0^pi cos(t - x sin t) dt
//                (9.1.21) by the trapezoid rule on 32 intervals; for this
//                periodic analytic integrand the rule is exact up to
//                J_65(x) - J_63(x), below 1e-18 here, and the two end terms
//                cancel (cos 0 + cos pi = 0);
//   x >= 25      Hankel's expansion (9.2.5, 9.2.9, 9.2.10) with mu = 4:
//                J1 = sqrt(2 / (pi x)) (P cos w - Q sin w), w = x - 3 pi / 4,
//                rewritten through sin x and cos x (exactly reduced by the
//                math library) as (P (sin x - cos x) + Q (sin x + cos x)) /
//                sqrt(pi x); the terms t_k = t_(k-1) (mu - (2k - 1)^2) / (8 k x)
//                fall for every k < 2x and are summed down to 1e-17.
// s_sin[j] = sin(j pi / 32).
__device__ double bessel_j1(double x, const double *s_sin) {
  if (x < 2.0) {
    const double q = -0.25 * x * x;
    double t = 0.5 * x, s = t;
    for (int m = 1; m <= 14; ++m) {
      t *= q / (double)(m * (m + 1));
      s += t;
    }
    return s;
  }
  if (x < 25.0) {
    double s = 0.0;
    for (int j = 1; j < 32; ++j) s += cos(j * (PI_D / 32.0) - x * s_sin[j]);
    return s * (1.0 / 32.0);
  }
  double P = 1.0, Q = 0.0, t = 1.0;
  const double inv8x = 0.125 / x;
  for (int k = 1; k <= 30; ++k) {
    const double f = (double)((2 * k - 1) * (2 * k - 1));
    t *= (4.0 - f) * inv8x / (double)k;
    // k = 1, 2, 3, 4, ... contributes +Q, -P, -Q, +P, ...
    const double sg = (((k + 1) >> 1) & 1) ? 1.0 : -1.0;
    if (k & 1) Q += sg * t; else P -= sg * t;
    if (fabs(t) < 1e-17) break;
  }
  double sx, cx;
  sincos(x, &sx, &cx);
  return (P * (sx - cx) + Q * (sx + cx)) / sqrt(PI_D * x);
}

// One block per chi node: threads stride over the window nodes, then a block
// reduction of the trapezoid sum.
__global__ __launch_bounds__(256) void k_sigma_w2(DevTables T, double theta, double *sw) {
  __shared__ double s_sin[32];
  __shared__ double part[256 / WAVE];
  if (threadIdx.x < 32) s_sin[threadIdx.x] = sin(threadIdx.x * (PI_D / 32.0));
  __syncthreads();
  const int n = blockIdx.x;
  const double chi = T.chi[n];
  const double *row = T.P + (size_t)n * T.n_k;
  const double l0 = log(T.k[0]), l1 = log(T.k[T.n_k - 1]);
  const double h = (l1 - l0) / (WINDOW_NODES - 1);
  double s = 0.0;
  for (int j = threadIdx.x; j < WINDOW_NODES; j += blockDim.x) {
    const double eps = j == 0 ? T.k[0] : (j == WINDOW_NODES - 1 ? T.k[T.n_k - 1] : exp(l0 + j * h));
    const double x = eps * chi * theta;
    const double win = bessel_j1(x, s_sin) / x;
    int jj;
    double t;
    if (!bracket_lnk(T.k, T.n_k, eps, jj, t)) continue;  // every node lies on the table
    const double P = exp((1.0 - t) * log(row[jj]) + t * log(row[jj + 1]));
    const double w = (j == 0 || j == WINDOW_NODES - 1) ? 0.5 * h : h;
    s += w * eps * eps * win * win * P;
  }
  s = wave_sum(s);
  if ((threadIdx.x & (WAVE - 1)) == 0) part[threadIdx.x / WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < 256 / WAVE; ++w) tot += part[w];
    sw[n] = 2.0 / PI_D * tot;
  }
}

void launch_sigma_w2(const DevTables &T, double theta, double *sw, hipStream_t s) {
  hipLaunchKernelGGL(k_sigma_w2, dim3((unsigned)T.n_chi), dim3(256), 0, s, T, theta, sw);
}

}  // namespace wlc
