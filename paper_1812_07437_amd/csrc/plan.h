// Internal plan representation shared by the host planner and the launchers.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/wlcov.h"

namespace wlc {

// One ell-configuration: a single ell-bin (power spectrum, used as the pair
// l, -l) or a binned triangle l1 <= l2 <= l3.
struct Config {
  int32_t kind;     // 2 or 3 legs
  int32_t leg[3];   // ell-bin of each leg (P: b, b, -1)
};

struct Plan {
  wlc_config cfg{};
  int n_ell_all = 0, n_ell = 0;             // bins in range, bins below ell_cut
  std::vector<double> edges, centres, widths;
  std::vector<Config> cfgs;                 // [n_ell] P configs, then triangles
  std::vector<int32_t> cfgT;                // [n_cfg][4]: kind, legs
  std::vector<int32_t> triT;                // [max(1, n_tri)][3]: legs of each triangle
  int n_tri = 0;
  // distinct (sorted) rows: cfg, z0, z1, z2
  std::vector<int32_t> rowR;                // [n_R][4]
  // output rows: cfg, e, z0, z1, z2, l0, l1, l2
  std::vector<int32_t> rowO;                // [n_out][8]
  int64_t n_R = 0, n_out = 0, n_p = 0;
  std::vector<double> n_modes, n_tri_closed; // closed-form counts
  std::vector<int64_t> lattice_thr;         // ceil((e_b/l_f)^2), [n_ell_all + 1]
  // bin averaging: n_sub equal sub-bins per used ell-bin; sub_centres
  // [n_ell * n_sub] (the bin centres when n_sub = 1), and per configuration
  // c the entries sub_off[c] .. sub_off[c + 1] - 1 of sub_leg [.][4] (the
  // sub-bin index of each leg, -1 where unused) and sub_w (weights, sum 1)
  int n_sub = 1;
  std::vector<double> sub_centres;
  std::vector<int32_t> sub_off, sub_leg;
  std::vector<double> sub_w;
  // rows in ell_max order (stable by the largest ell-bin of their legs) and,
  // per used bin b, the number of rows whose largest bin is <= b
  std::vector<int32_t> lmax_perm;
  std::vector<int32_t> lmax_ends;
  double omega = 0.0;                       // 4 pi f_sky
  double noise = 0.0;                       // sigma_eps^2 / n_i
  // Flattened Gram products (every precision but FP64_CHI): the rows of A in
  // order of their lowest redshift bin (stable), so that the rows whose
  // lensing kernels end earliest share panels; arow [r_pad] is the distinct
  // row of each A-row (-1 past n_R), pos [n_R] its inverse.  Empty for
  // FP64_CHI.
  std::vector<int32_t> arow, pos;
  // sizes
  int64_t k_len = 0, k_pad = 0, r_pad = 0, n_pad = 0;
  size_t ws_run = 0, ws_snr = 0;
};

// Precision modes: valid range, and whether the covariance (and the Gram
// output) is FP64.
inline bool prec_valid(int p) { return p >= WLC_FP64 && p <= WLC_BF16_AUTO; }
inline bool prec_f64(int p) { return p == WLC_FP64 || p == WLC_FP64_CHI; }

void set_error(const std::string &msg);
const char *last_error();
int fail(int code, const std::string &msg);

// Enumerate everything; returns WLC_OK or an error code (message set).
int build_plan(const wlc_config &cfg, Plan &p);

}  // namespace wlc
