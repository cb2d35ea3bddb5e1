// Host planner: ell-bins, triangles, tomographic rows and the distinct-row map.
//
// Follows Rizzato et al. (2019), arXiv 1812.07437: log-spaced ell-bins whose
// centre is the middle of the bin (Sec. 3.2.1, App. A); triangles
// l1 <= l2 <= l3 with j fastest and k slowest (Sec. 5); tomographic pairs
// i <= j with j fastest and bispectrum triplets with k fastest (Sec. 5), all
// n^3 combinations for scalene triangles and one ordering of the bins on
// equal sides.  Under Limber every bin sees the same chi, so a row's value
// depends only on its ell-configuration and the multiset of its bins; each
// row maps to the row holding the sorted multiset ("distinct" rows).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>

#include "plan.h"

namespace wlc {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }
const char *last_error() { return g_err.c_str(); }
int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

static inline int64_t rank_pair(int n, int i, int j) {  // i <= j
  return (int64_t)i * n - (int64_t)i * (i - 1) / 2 + (j - i);
}

int build_plan(const wlc_config &c, Plan &p) {
  if (c.n_z < 1 || c.n_ell < 1 || c.n_chi < 1 || c.n_k < 2 || c.n_m < 1)
    return fail(WLC_EINVAL, "n_z, n_ell, n_chi, n_m must be >= 1 and n_k >= 2");
  if (c.n_z > 64) return fail(WLC_EINVAL, "n_z must be <= 64");
  if (!(c.ell_min > 0.0) || !(c.ell_max > c.ell_min) || !std::isfinite(c.ell_max))
    return fail(WLC_EINVAL, "need 0 < ell_min < ell_max");
  if (!(c.f_sky > 0.0 && c.f_sky <= 1.0)) return fail(WLC_EINVAL, "f_sky must be in (0, 1]");
  if (!(c.sigma_eps >= 0.0) || !(c.n_gal_arcmin2 > 0.0) || !(c.sigma_b2 >= 0.0) || !(c.k_max > 0.0) ||
      !(c.rho_mean > 0.0))
    return fail(WLC_EINVAL, "survey scalars must be finite and positive");
  if (c.tomo_mode != WLC_TOMO_PAPER && c.tomo_mode != WLC_TOMO_SORTED)
    return fail(WLC_EINVAL, "unknown tomo_mode");
  if (!prec_valid(c.precision)) return fail(WLC_EINVAL, "unknown precision");
  p.cfg = c;
  const int nz = c.n_z;

  // ell-bins: e_b = exp(ln l_min + b (ln l_max - ln l_min) / n)
  p.n_ell_all = c.n_ell;
  const double a = std::log(c.ell_min), b = std::log(c.ell_max);
  p.edges.resize(c.n_ell + 1);
  for (int i = 0; i <= c.n_ell; ++i) p.edges[i] = std::exp(a + i * (b - a) / c.n_ell);
  p.centres.resize(c.n_ell);
  p.widths.resize(c.n_ell);
  for (int i = 0; i < c.n_ell; ++i) {
    p.centres[i] = (p.edges[i] + p.edges[i + 1]) / 2.0;
    p.widths[i] = p.edges[i + 1] - p.edges[i];
  }
  p.n_ell = c.n_ell;
  if (c.ell_cut > 0.0) {
    p.n_ell = 0;
    for (int i = 0; i < c.n_ell; ++i)
      if (p.centres[i] < c.ell_cut) ++p.n_ell;
    if (p.n_ell == 0) return fail(WLC_EINVAL, "ell_cut removes every ell-bin");
  }
  const int nl = p.n_ell;

  // configurations: P bins, then triangles in data-vector order
  p.cfgs.clear();
  for (int i = 0; i < nl; ++i) p.cfgs.push_back(Config{2, {i, i, -1}});
  for (int k = 0; k < nl; ++k)
    for (int i = 0; i <= k; ++i)
      for (int j = i; j <= k; ++j)
        if (p.centres[i] + p.centres[j] > p.centres[k]) p.cfgs.push_back(Config{3, {i, j, k}});
  p.n_tri = (int)p.cfgs.size() - nl;
  p.cfgT.assign(p.cfgs.size() * 4, 0);
  for (size_t q = 0; q < p.cfgs.size(); ++q) {
    p.cfgT[4 * q] = p.cfgs[q].kind;
    for (int a = 0; a < 3; ++a) p.cfgT[4 * q + 1 + a] = p.cfgs[q].leg[a];
  }
  p.triT.assign((size_t)std::max(1, p.n_tri) * 3, 0);
  for (int t = 0; t < p.n_tri; ++t)
    for (int a = 0; a < 3; ++a) p.triT[3 * t + a] = p.cfgs[nl + t].leg[a];

  // distinct rows: P pairs i <= j, B triplets i <= j <= k
  const int64_t npair = (int64_t)nz * (nz + 1) / 2;
  const int64_t ntrip = (int64_t)nz * (nz + 1) * (nz + 2) / 6;
  std::vector<int64_t> trip_rank((size_t)nz * nz * nz, -1);
  {
    int64_t q = 0;
    for (int i = 0; i < nz; ++i)
      for (int j = i; j < nz; ++j)
        for (int k = j; k < nz; ++k) trip_rank[((size_t)i * nz + j) * nz + k] = q++;
  }
  p.rowR.clear();
  for (int l = 0; l < nl; ++l)
    for (int i = 0; i < nz; ++i)
      for (int j = i; j < nz; ++j) {
        int32_t r[4] = {l, i, j, -1};
        p.rowR.insert(p.rowR.end(), r, r + 4);
      }
  for (int t = 0; t < p.n_tri; ++t)
    for (int i = 0; i < nz; ++i)
      for (int j = i; j < nz; ++j)
        for (int k = j; k < nz; ++k) {
          int32_t r[4] = {nl + t, i, j, k};
          p.rowR.insert(p.rowR.end(), r, r + 4);
        }
  p.n_R = (int64_t)p.rowR.size() / 4;

  // output rows in the data-vector order
  p.rowO.clear();
  for (int l = 0; l < nl; ++l)
    for (int i = 0; i < nz; ++i)
      for (int j = i; j < nz; ++j) {
        int32_t e = (int32_t)(l * npair + rank_pair(nz, i, j));
        int32_t r[8] = {l, e, i, j, -1, l, l, -1};
        p.rowO.insert(p.rowO.end(), r, r + 8);
      }
  p.n_p = (int64_t)nl * npair;
  for (int t = 0; t < p.n_tri; ++t) {
    const Config &cf = p.cfgs[nl + t];
    const int l1 = cf.leg[0], l2 = cf.leg[1], l3 = cf.leg[2];
    for (int i = 0; i < nz; ++i)
      for (int j = 0; j < nz; ++j)
        for (int k = 0; k < nz; ++k) {
          bool keep;
          if (c.tomo_mode == WLC_TOMO_SORTED) keep = (i <= j && j <= k);
          else if (l1 != l2 && l2 != l3) keep = true;            // scalene
          else if (l1 == l2 && l2 == l3) keep = (i <= j && j <= k);  // equilateral
          else if (l1 == l2) keep = (i <= j);                     // l1 = l2 < l3
          else keep = (j <= k);                                   // l1 < l2 = l3
          if (!keep) continue;
          int s[3] = {i, j, k};
          if (s[0] > s[1]) std::swap(s[0], s[1]);
          if (s[1] > s[2]) std::swap(s[1], s[2]);
          if (s[0] > s[1]) std::swap(s[0], s[1]);
          int64_t e = p.n_p + (int64_t)t * ntrip + trip_rank[((size_t)s[0] * nz + s[1]) * nz + s[2]];
          int32_t r[8] = {nl + t, (int32_t)e, i, j, k, l1, l2, l3};
          p.rowO.insert(p.rowO.end(), r, r + 8);
        }
  }
  p.n_out = (int64_t)p.rowO.size() / 8;
  if (p.n_out > (int64_t)std::numeric_limits<int32_t>::max() / 2)
    return fail(WLC_EINVAL, "data vector too long");

  // closed-form counts (Sec. 3.2.2, App. B)
  p.omega = 4.0 * M_PI * c.f_sky;
  p.n_modes.resize(nl);
  for (int i = 0; i < nl; ++i) p.n_modes[i] = 2.0 * p.centres[i] * p.widths[i] * c.f_sky;
  p.n_tri_closed.resize(p.n_tri);
  for (int t = 0; t < p.n_tri; ++t) {
    const Config &cf = p.cfgs[nl + t];
    const double l1 = p.centres[cf.leg[0]], l2 = p.centres[cf.leg[1]], l3 = p.centres[cf.leg[2]];
    const double d1 = p.widths[cf.leg[0]], d2 = p.widths[cf.leg[1]], d3 = p.widths[cf.leg[2]];
    const double lam2 = 2 * l1 * l1 * l2 * l2 + 2 * l1 * l1 * l3 * l3 + 2 * l2 * l2 * l3 * l3 -
                        l1 * l1 * l1 * l1 - l2 * l2 * l2 * l2 - l3 * l3 * l3 * l3;
    if (!(lam2 > 0.0)) return fail(WLC_EINVAL, "degenerate (flat) binned triangle");
    p.n_tri_closed[t] = p.omega * p.omega * l1 * l2 * l3 * d1 * d2 * d3 / (2.0 * M_PI * M_PI * M_PI * std::sqrt(lam2));
  }
  // lattice thresholds, l_f = 2 pi / sqrt(Omega)
  const double lf = 2.0 * M_PI / std::sqrt(p.omega);
  p.lattice_thr.resize(c.n_ell + 1);
  for (int i = 0; i <= c.n_ell; ++i) p.lattice_thr[i] = (int64_t)std::ceil((p.edges[i] / lf) * (p.edges[i] / lf));

  // shot noise per bin: sigma_eps^2 / (n_gal / n_z) with n_gal per steradian
  const double arcmin2_per_sr = (10800.0 / M_PI) * (10800.0 / M_PI);
  p.noise = c.sigma_eps * c.sigma_eps / (c.n_gal_arcmin2 * arcmin2_per_sr / nz);
  (void)ntrip;
  return WLC_OK;
}

}  // namespace wlc
