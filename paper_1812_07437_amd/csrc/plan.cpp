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

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n).
static void gauss_legendre(int n, double *x, double *w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Continuum number of ordered pairs (l1, l2) of 2-D modes with |l1| in
// [a1, b1), |l2| in [a2, b2) and |l1 + l2| in [a3, b3), up to the constant
// (Omega / (2 pi)^2)^2 2 pi (App. B: N_tri as the sum of the selection
// function): int int l1 l2 dphi(l1, l2) dl1 dl2, where dphi is the measure
// of the angles phi between the two modes with l1^2 + l2^2 + 2 l1 l2 cos
// phi in [a3^2, b3^2), by Gauss-Legendre on 8 x 8 nodes.
static double cell_count(double a1, double b1, double a2, double b2, double a3, double b3) {
  double x[8], w[8];
  gauss_legendre(8, x, w);
  double s = 0.0;
  for (int i = 0; i < 8; ++i) {
    const double l1 = 0.5 * (a1 + b1) + 0.5 * (b1 - a1) * x[i], w1 = 0.5 * (b1 - a1) * w[i];
    for (int j = 0; j < 8; ++j) {
      const double l2 = 0.5 * (a2 + b2) + 0.5 * (b2 - a2) * x[j], w2 = 0.5 * (b2 - a2) * w[j];
      const double clo = std::min(1.0, std::max(-1.0, (a3 * a3 - l1 * l1 - l2 * l2) / (2.0 * l1 * l2)));
      const double chi = std::min(1.0, std::max(-1.0, (b3 * b3 - l1 * l1 - l2 * l2) / (2.0 * l1 * l2)));
      s += w1 * w2 * l1 * l2 * 2.0 * (std::acos(clo) - std::acos(chi));
    }
  }
  return s;
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
  if (c.n_sub < 0 || c.n_sub > 8) return fail(WLC_EINVAL, "n_sub must be in 0..8");
  if (c.n_sub > 1 && (c.flags & WLC_FLAG_NGINS))
    return fail(WLC_EINVAL, "bin averaging (n_sub > 1) does not cover the B.B, P.T and P.B terms");
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

  // ell_max order (eq. eq:SN): the data vector cut at an ell_max between
  // bins b and b + 1 is the set of rows whose legs all lie in bins <= b, so
  // with rows sorted by their largest bin every cut is a leading block
  {
    std::vector<int32_t> top((size_t)p.n_out);
    for (int64_t a = 0; a < p.n_out; ++a) {
      const int32_t *r = &p.rowO[8 * a];
      top[a] = std::max(r[5], std::max(r[6], r[7]));
    }
    p.lmax_perm.resize((size_t)p.n_out);
    for (int64_t a = 0; a < p.n_out; ++a) p.lmax_perm[a] = (int32_t)a;
    std::stable_sort(p.lmax_perm.begin(), p.lmax_perm.end(), [&](int32_t x, int32_t y) { return top[x] < top[y]; });
    p.lmax_ends.assign(nl, 0);
    for (int64_t a = 0; a < p.n_out; ++a)
      for (int b = top[a]; b < nl; ++b) ++p.lmax_ends[b];
  }

  // bin averaging: sub-bins of equal width; a power-spectrum bin averages
  // over its sub-bins with weights proportional to their number of modes
  // (2 l dl f_sky, Sec. 3.2.2), a triangle bin over the cells of sub-bin
  // triples whose centres obey the strict triangle inequality, weighted by
  // the continuum count of triangles in the cell (App. B)
  const int S = c.n_sub > 1 ? c.n_sub : 1;
  p.n_sub = S;
  p.sub_centres.resize((size_t)nl * S);
  for (int i = 0; i < nl; ++i)
    for (int s = 0; s < S; ++s)
      p.sub_centres[(size_t)i * S + s] = S == 1 ? p.centres[i] : p.edges[i] + (s + 0.5) * p.widths[i] / S;
  p.sub_off.assign(p.cfgs.size() + 1, 0);
  p.sub_leg.clear();
  p.sub_w.clear();
  for (size_t q = 0; q < p.cfgs.size(); ++q) {
    const Config &cf = p.cfgs[q];
    const size_t first = p.sub_w.size();
    double wsum = 0.0;
    if (S == 1) {
      int32_t e[4] = {cf.leg[0], cf.leg[1], cf.leg[2], -1};
      p.sub_leg.insert(p.sub_leg.end(), e, e + 4);
      p.sub_w.push_back(1.0);
    } else if (cf.kind == 2) {
      for (int s = 0; s < S; ++s) {
        const int32_t g = cf.leg[0] * S + s;
        int32_t e[4] = {g, g, -1, -1};
        p.sub_leg.insert(p.sub_leg.end(), e, e + 4);
        p.sub_w.push_back(p.sub_centres[g]);
        wsum += p.sub_centres[g];
      }
    } else {
      for (int s1 = 0; s1 < S; ++s1)
        for (int s2 = 0; s2 < S; ++s2)
          for (int s3 = 0; s3 < S; ++s3) {
            const int32_t g1 = cf.leg[0] * S + s1, g2 = cf.leg[1] * S + s2, g3 = cf.leg[2] * S + s3;
            const double l1 = p.sub_centres[g1], l2 = p.sub_centres[g2], l3 = p.sub_centres[g3];
            if (!(l1 < l2 + l3 && l2 < l1 + l3 && l3 < l1 + l2)) continue;
            const double h1 = p.widths[cf.leg[0]] / S, h2 = p.widths[cf.leg[1]] / S, h3 = p.widths[cf.leg[2]] / S;
            const double rho = cell_count(l1 - 0.5 * h1, l1 + 0.5 * h1, l2 - 0.5 * h2, l2 + 0.5 * h2,
                                          l3 - 0.5 * h3, l3 + 0.5 * h3);
            if (!(rho > 0.0)) continue;
            int32_t e[4] = {g1, g2, g3, -1};
            p.sub_leg.insert(p.sub_leg.end(), e, e + 4);
            p.sub_w.push_back(rho);
            wsum += rho;
          }
      if (p.sub_w.size() == first) return fail(WLC_EINVAL, "a binned triangle has no sub-bin triangle");
    }
    if (S > 1)
      for (size_t e = first; e < p.sub_w.size(); ++e) p.sub_w[e] /= wsum;
    p.sub_off[q + 1] = (int32_t)p.sub_w.size();
  }

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
