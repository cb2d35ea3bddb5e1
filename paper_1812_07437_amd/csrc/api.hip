// C ABI of libwlcov: plans, workspace layout and the launch sequence of the
// hot path (see include/wlcov.h for the contract of every entry point).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "engine.h"

struct wlc_plan_s {
  wlc::Plan p;
  // phase timing (HIP events recorded on the run's stream)
  bool timing = false;
  bool events_ready = false;
  bool recorded[WLC_PHASE_COUNT] = {};
  hipEvent_t ev[2 * WLC_PHASE_COUNT] = {};
  // per-launch events of the Cholesky block-update kernel
  std::vector<hipEvent_t> upd_ev;
  wlc::KernelProbe probe;
  bool probe_valid = false;
  ~wlc_plan_s() {
    if (events_ready)
      for (auto &e : ev) (void)hipEventDestroy(e);
    for (auto &e : upd_ev) (void)hipEventDestroy(e);
  }
};

namespace {
struct PlanTimer : wlc::PhaseHooks {
  wlc_plan_s *h;
  hipStream_t s;
  PlanTimer(wlc_plan_s *h_, hipStream_t s_) : h(h_), s(s_) {}
  void begin(int ph) override { (void)hipEventRecord(h->ev[2 * ph], s); }
  void end(int ph) override {
    (void)hipEventRecord(h->ev[2 * ph + 1], s);
    h->recorded[ph] = true;
  }
};
}  // namespace

namespace wlc {

static inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
static inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

constexpr int64_t GRAM_TILE = 256;  // rows of A padded to the bf16 Gram tile
constexpr int64_t K_ALIGN = 64;

enum Buf {
  B_ROWR, B_ROWO, B_CFGT, B_CENT, B_NMODES, B_NTRI, B_THR, B_TRI, B_FLAGS,
  B_U, B_PK, B_NE, B_X, B_R, B_DR, B_RR, B_PS, B_G, B_GMAX, B_TS, B_SEXP,
  B_A0, B_A1, B_GM, B_PART, B_H, B_G2, B_H2, B_TS2, B_T2, B_SW, B_SOFF, B_SLEG, B_SWT, B_SQ, B_GD, B_FP,
  B_AROW, B_POS, B_EXT, B_GP, NBUF
};

// Columns per chi node of the configuration factor G: the mass nodes, and
// with the chi-resolved super-sample term one more.
static int g_cols(const wlc_config &c) { return c.n_m + ((c.flags & WLC_FLAG_SSC_CHI) ? 1 : 0); }
// Angular radius of the survey: Omega = 2 pi (1 - cos Theta) (Sec. 3.2.2).
static double theta_sky(const Plan &p) { return std::acos(1.0 - p.omega / (2.0 * 3.14159265358979323846)); }

// two-leg trispectrum (B.B / P.T / P.B terms): configurations and rows
static int twoleg_configs(const Plan &p) { return p.n_ell + p.n_ell * (p.n_ell - 1) / 2; }
static int64_t twoleg_rows(const Plan &p) {
  const int nz = p.cfg.n_z;
  return (int64_t)p.n_ell * (nz * (nz + 1) / 2) + (int64_t)(twoleg_configs(p) - p.n_ell) * nz * nz;
}
static int64_t twoleg_ld(const Plan &p) { return round_up(twoleg_rows(p), 64); }

struct Layout {
  size_t off[NBUF];
  size_t total;
};

static Layout run_layout(const Plan &p) {
  const auto &c = p.cfg;
  size_t sz[NBUF] = {};
  const int64_t n_cfg = (int64_t)p.cfgs.size();
  const int nl = p.n_ell;
  sz[B_ROWR] = p.rowR.size() * 4;
  sz[B_ROWO] = p.rowO.size() * 4;
  sz[B_CFGT] = (size_t)n_cfg * 16;
  const size_t n_ls = (size_t)nl * p.n_sub;  // staged ell values: bin centres or sub-bins
  sz[B_CENT] = n_ls * 8;
  sz[B_NMODES] = (size_t)nl * 8;
  sz[B_NTRI] = (size_t)std::max(1, p.n_tri) * 8;
  sz[B_THR] = p.lattice_thr.size() * 8;
  sz[B_TRI] = (size_t)std::max(1, p.n_tri) * 12;
  sz[B_FLAGS] = 64 * 4;
  sz[B_U] = n_ls * c.n_chi * c.n_m * 8;
  sz[B_PK] = sz[B_NE] = n_ls * c.n_chi * 8;
  sz[B_X] = sz[B_R] = (size_t)n_cfg * c.n_chi * 8;
  sz[B_DR] = sz[B_RR] = (size_t)p.n_R * 8;
  sz[B_PS] = (size_t)nl * c.n_z * c.n_z * 8;
  sz[B_G] = (size_t)n_cfg * c.n_chi * g_cols(c) * 8;
  sz[B_GMAX] = (size_t)n_cfg * c.n_chi * 8;
  sz[B_TS] = (size_t)p.n_R * c.n_chi * 8;
  sz[B_SEXP] = (size_t)p.n_R * 4;
  const bool chi = c.precision == WLC_FP64_CHI;
  const size_t ael = c.precision == WLC_FP64 ? 8 : (c.precision == WLC_FP32 ? 4 : 2);
  sz[B_A0] = chi ? 0 : (size_t)p.r_pad * p.k_pad * ael;
  sz[B_A1] = c.precision == WLC_BF16X3 || c.precision == WLC_BF16_AUTO ? sz[B_A0] : 0;
  if (!p.arow.empty()) {  // A-rows in their own order: index maps, panel extents, the product in that order
    sz[B_AROW] = p.arow.size() * 4;
    sz[B_POS] = p.pos.size() * 4;
    sz[B_EXT] = (size_t)(p.r_pad / GRAM_TILE) * 4;
    sz[B_GP] = (size_t)p.r_pad * p.r_pad * (c.precision == WLC_FP64 ? 8 : 4);
  }
  if (c.precision == WLC_BF16_AUTO) {  // the per-tile precision plan
    sz[B_SQ] = (size_t)n_cfg * c.n_chi * 8;
    sz[B_GD] = (size_t)p.n_R * 8;
    sz[B_FP] = (size_t)(p.r_pad / GRAM_TILE + 1) * 8;  // per panel, then the largest
  }
  const size_t gel = prec_f64(c.precision) ? 8 : 4;
  sz[B_GM] = (size_t)p.r_pad * p.r_pad * gel;
  GramShape g{p.r_pad, p.k_pad, p.r_pad, p.k_pad};
  sz[B_PART] = chi ? 0 : gram_partial_bytes(c.precision, g);
  sz[B_H] = chi ? (size_t)n_cfg * n_cfg * c.n_chi * 8 : 0;
  if (c.flags & WLC_FLAG_NGINS) {
    const int n2 = twoleg_configs(p);
    sz[B_G2] = (size_t)n2 * c.n_chi * c.n_m * 8;
    sz[B_H2] = (size_t)n2 * n2 * c.n_chi * 8;
    sz[B_TS2] = (size_t)twoleg_rows(p) * c.n_chi * 8;
    sz[B_T2] = (size_t)twoleg_rows(p) * twoleg_ld(p) * 8;
  }
  if (c.flags & WLC_FLAG_SSC_CHI) sz[B_SW] = (size_t)c.n_chi * 8;
  sz[B_SOFF] = p.sub_off.size() * 4;
  sz[B_SLEG] = p.sub_leg.size() * 4;
  sz[B_SWT] = p.sub_w.size() * 8;
  Layout L{};
  size_t o = 0;
  for (int b = 0; b < NBUF; ++b) {
    L.off[b] = o;
    o = align_up(o + sz[b], 256);
  }
  L.total = o;
  return L;
}

static int64_t snr_ld(int64_t n) { return round_up(n + 1, 8); }

size_t run_ws_bytes(const Plan &p) { return run_layout(p).total; }

size_t snr_ws_bytes(const Plan &p) {
  const int64_t n = p.n_out, ld = snr_ld(n);
  // bordered matrix, Cholesky scratch, flag, result; then the ell_max order,
  // its group ends, group sums and the curve (wlc_snr2_lmax)
  return align_up((size_t)(n + 1) * ld * 8, 256) + align_up(chol_scratch_bytes(n), 256) + 256 + 256 +
         align_up((size_t)n * 4, 256) + 3 * align_up((size_t)p.n_ell * 8, 256);
}

// PCA workspace: the S/N workspace (bordered Cholesky), then X and V
// [n_pad][n_pad], y [n_pad], per-mode arrays and the convergence word.
static int64_t pca_pad(const Plan &p) { return round_up(p.n_out, 64); }
// Jacobi sweeps on each pair's 64 x 64 Gram matrix per round: one sweep
// measured as fast in outer sweeps as full diagonalisation, at a third of
// the cost.
constexpr int PCA_INNER = 1;

size_t pca_ws_bytes(const Plan &p) {
  const int64_t np = pca_pad(p), n = p.n_out;
  if (np > 65535) return 0;
  const size_t pairs = (size_t)np / 64;
  return align_up(snr_ws_bytes(p), 256) + 2 * align_up((size_t)np * np * 8, 256) + align_up((size_t)np * 8, 256) +
         5 * align_up((size_t)n * 8, 256) + 2 * align_up((size_t)n * 4, 256) + 256 +
         align_up(pairs * pca_slices(np) * 64 * 64 * 8, 256) + align_up(pairs * 64 * 64 * 8, 256) +
         align_up(pairs * 4, 256);
}

size_t snr_structured_ws_bytes(const Plan &p) {
  if (p.cfg.tomo_mode != WLC_TOMO_PAPER || p.cfg.n_z > WOOD_NZ_MAX || (p.cfg.flags & WLC_FLAG_NGINS)) return 0;
  const int64_t n = p.n_R, ldw = snr_ld(n), ldt = round_up(n, 8);
  const int nz = p.cfg.n_z, sp = nz * (nz + 1) / 2, sb = nz * (nz + 1) * (nz + 2) / 6;
  const size_t blocks = (size_t)p.n_ell * sp * sp + (size_t)p.n_tri * sb * sb;
  return align_up((size_t)(n + 1) * ldw * 8, 256) + align_up((size_t)n * ldt * 8, 256) + align_up(blocks * 8, 256) +
         align_up((size_t)p.n_ell * nz * nz * 8, 256) + align_up((size_t)n * 4, 256) + align_up((size_t)n * 8, 256) +
         align_up(chol_scratch_bytes(n), 256) + 256 + 256;
}

// The A-row order of the flattened one-halo products: distinct rows by their lowest
// redshift bin (rows hold their bins in increasing order), stably.  The
// factor of a row vanishes beyond the far edge of its lowest bin (eq.
// KernelLensing1: W_i(chi) = 0 past the sources of bin i), so panels of rows
// with the same lowest bin end at the same chi node, and a tile's product
// stops where the shorter of its two panels ends.
static void order_arows(Plan &p) {
  p.arow.clear();
  p.pos.clear();
  const int prec = p.cfg.precision;
  if (prec == WLC_FP64_CHI) return;  // no flattened product
  const int nz = p.cfg.n_z;
  std::vector<int64_t> start((size_t)nz + 1, 0);
  for (int64_t e = 0; e < p.n_R; ++e) ++start[(size_t)p.rowR[4 * e + 1] + 1];
  for (int z = 0; z < nz; ++z) start[(size_t)z + 1] += start[(size_t)z];
  p.arow.assign((size_t)p.r_pad, -1);
  p.pos.assign((size_t)p.n_R, 0);
  for (int64_t e = 0; e < p.n_R; ++e) {
    const int64_t r = start[(size_t)p.rowR[4 * e + 1]]++;
    p.arow[(size_t)r] = (int32_t)e;
    p.pos[(size_t)e] = (int32_t)r;
  }
}

static void finish_sizes(Plan &p) {
  p.k_len = (int64_t)p.cfg.n_chi * g_cols(p.cfg);
  p.k_pad = round_up(p.k_len, K_ALIGN);
  p.r_pad = round_up(p.n_R, GRAM_TILE);
  order_arows(p);
  p.ws_run = run_ws_bytes(p);
  p.ws_snr = snr_ws_bytes(p);
}

int snr_structured_enqueue(const Plan &p, const void *ws_run, void *ws, hipStream_t s, PhaseHooks *hooks,
                           KernelProbe *probe, int32_t **flag_dev, double **out_dev) {
  if (p.cfg.tomo_mode != WLC_TOMO_PAPER)
    return fail(WLC_EINVAL, "the structured S/N needs PAPER tomography (with SORTED rows use wlc_snr2)");
  if (p.cfg.n_z > WOOD_NZ_MAX) return fail(WLC_EINVAL, "the structured S/N supports at most 32 redshift bins");
  if (p.cfg.flags & WLC_FLAG_NGINS)
    return fail(WLC_EINVAL, "the structured S/N does not cover the B.B, P.T and P.B terms (WLC_FLAG_NGINS)");
  const Layout L = run_layout(p);
  const wlc_config &c = p.cfg;
  const int64_t n = p.n_R, ldw = snr_ld(n), ldt = round_up(n, 8);
  const int nz = c.n_z, sp = nz * (nz + 1) / 2, sb = nz * (nz + 1) * (nz + 2) / 6;
  const size_t blocks = (size_t)p.n_ell * sp * sp + (size_t)p.n_tri * sb * sb;
  char *base = static_cast<char *>(ws);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char *q = base + o;
    o += align_up(bytes, 256);
    return q;
  };
  WoodArgs w{};
  w.W = reinterpret_cast<double *>(take((size_t)(n + 1) * ldw * 8));
  w.ld_w = ldw;
  w.T = reinterpret_cast<double *>(take((size_t)n * ldt * 8));
  w.ld_t = ldt;
  w.Gb = reinterpret_cast<double *>(take(blocks * 8));
  w.Q = reinterpret_cast<double *>(take((size_t)p.n_ell * nz * nz * 8));
  w.tau = reinterpret_cast<int32_t *>(take((size_t)n * 4));
  w.rhat = reinterpret_cast<double *>(take((size_t)n * 8));
  double *scratch = reinterpret_cast<double *>(take(chol_scratch_bytes(n)));
  int32_t *flag = reinterpret_cast<int32_t *>(take(256));
  double *out = reinterpret_cast<double *>(take(256));
  w.B = BlockMap{p.n_ell, p.n_tri, sp, sb, n};
  w.n_ell = p.n_ell;
  w.nz = nz;
  const void *wr = ws_run;
  auto run_at = [&](Buf b) { return static_cast<const char *>(wr) + L.off[b]; };
  w.Ps = reinterpret_cast<const double *>(run_at(B_PS));
  w.nmodes = reinterpret_cast<const double *>(run_at(B_NMODES));
  w.ntri = reinterpret_cast<const double *>(run_at(B_NTRI));
  w.dR = reinterpret_cast<const double *>(run_at(B_DR));
  w.rR = reinterpret_cast<const double *>(run_at(B_RR));
  w.cfgT = reinterpret_cast<const int32_t *>(run_at(B_CFGT));
  w.sexp = reinterpret_cast<const int32_t *>(run_at(B_SEXP));
  w.Gm = run_at(B_GM);
  w.gm_f32 = !prec_f64(c.precision);
  w.ld_g = p.r_pad;
  w.omega = p.omega;
  w.sigma_b2 = (c.flags & WLC_FLAG_SSC_CHI) ? 0.0 : c.sigma_b2;  // else inside the Gram product
  w.flag = flag;
  if (hooks) hooks->begin(WLC_PHASE_SNR_PREP);
  launch_fill_i32(flag, 1, 0, s);
  launch_woodbury(w, s);
  if (hooks) hooks->end(WLC_PHASE_SNR_PREP);
  if (hooks) hooks->begin(WLC_PHASE_CHOL);
  chol_factor(w.W, n, ldw, scratch, flag, s, probe);
  launch_sumsq_row(w.W, n, ldw, out, s);
  if (hooks) hooks->end(WLC_PHASE_CHOL);
  *flag_dev = flag;
  *out_dev = out;
  return hip_check(hipGetLastError(), "structured snr launch");
}

int hip_check(hipError_t e, const char *what) {
  if (e == hipSuccess) return WLC_OK;
  return fail(WLC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

__global__ void k_fill_i32(int32_t *p, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

void launch_fill_i32(int32_t *p, int n, int32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
}

__global__ void k_scale(const double *x, double *y, int64_t n, double a) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}

void launch_scale(const double *x, double *y, int64_t n, double a, hipStream_t s) {
  const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_scale, dim3(g), dim3(256), 0, s, x, y, n, a);
}

template <typename T>
static T *at(void *ws, const Layout &L, Buf b) {
  return reinterpret_cast<T *>(static_cast<char *>(ws) + L.off[b]);
}

struct Upload { Buf b; const void *src; size_t bytes; };

static int upload(const Upload *ups, size_t n, void *ws, const Layout &L, hipStream_t s) {
  for (size_t i = 0; i < n; ++i) {
    const Upload &u = ups[i];
    if (!u.bytes) continue;
    int rc = hip_check(hipMemcpyAsync(at<char>(ws, L, u.b), u.src, u.bytes, hipMemcpyHostToDevice, s),
                       "index upload");
    if (rc) return rc;
  }
  return WLC_OK;
}

// Copy the plan's index tables into the workspace (the sources live in the
// plan, which outlives every run using it).
static int upload_index(const Plan &p, void *ws, const Layout &L, hipStream_t s) {
  const Upload ups[] = {
      {B_ROWR, p.rowR.data(), p.rowR.size() * 4},
      {B_ROWO, p.rowO.data(), p.rowO.size() * 4},
      {B_CFGT, p.cfgT.data(), p.cfgT.size() * 4},
      {B_CENT, p.sub_centres.data(), p.sub_centres.size() * 8},
      {B_SOFF, p.sub_off.data(), p.sub_off.size() * 4},
      {B_SLEG, p.sub_leg.data(), p.sub_leg.size() * 4},
      {B_SWT, p.sub_w.data(), p.sub_w.size() * 8},
      {B_NMODES, p.n_modes.data(), p.n_modes.size() * 8},
      {B_NTRI, p.n_tri_closed.data(), p.n_tri_closed.size() * 8},
      {B_THR, p.lattice_thr.data(), p.lattice_thr.size() * 8},
      {B_TRI, p.triT.data(), p.triT.size() * 4},
      {B_AROW, p.arow.data(), p.arow.size() * 4},
      {B_POS, p.pos.data(), p.pos.size() * 4},
  };
  return upload(ups, sizeof(ups) / sizeof(ups[0]), ws, L, s);
}

static DevTables dev_tables(const Plan &p, const wlc_tables &tb, double rho = 0.0) {
  const wlc_config &c = p.cfg;
  return DevTables{tb.chi, tb.w_chi, tb.k, tb.m, tb.w_m, tb.W, tb.P, tb.u, tb.n_m, tb.b1, tb.b2,
                   c.n_z, c.n_chi, c.n_k, c.n_m, rho > 0.0 ? rho : c.rho_mean, c.k_max};
}

static int check_tables_present(const wlc_tables &tb) {
  if (!tb.chi || !tb.w_chi || !tb.k || !tb.m || !tb.w_m || !tb.W || !tb.P || !tb.u || !tb.n_m)
    return fail(WLC_EINVAL, "missing table");
  return WLC_OK;
}

int validate_tables(const Plan &p, const wlc_tables &tb, void *ws, hipStream_t s) {
  int rc = check_tables_present(tb);
  if (rc) return rc;
  const Layout L = run_layout(p);
  rc = upload_index(p, ws, L, s);
  if (rc) return rc;
  const DevTables T = dev_tables(p, tb);
  int32_t *flags = at<int32_t>(ws, L, B_FLAGS);
  launch_fill_i32(flags, 64, 0, s);
  launch_validate(T, at<double>(ws, L, B_CENT), p.n_ell * p.n_sub, (p.cfg.flags & WLC_FLAG_SSC_CHI) ? theta_sky(p) : 0.0,
                  flags, s);
  int32_t hf[3] = {0, 0, 0};
  rc = hip_check(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s), "validation copy");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "validation sync");
  if (rc) return rc;
  if (hf[0]) return fail(WLC_EINVAL, "tables must be finite, positive where required, and grids increasing");
  if (hf[1]) return fail(WLC_ERANGE, "the k table does not cover every ell/chi below k_max");
  if (hf[2]) return fail(WLC_ERANGE, "the k table must start below 0.1 / (chi_max Theta) for sigma_W^2");
  return WLC_OK;
}

static AsmArgs asm_args(const Plan &p, void *ws, const Layout &L);
static double split_lim(const Plan &p);

int run_enqueue_front(const Plan &p, const wlc_tables &tb, void *ws, hipStream_t s, PhaseHooks *hooks, double rho) {
  int rc = check_tables_present(tb);
  if (rc) return rc;
  const wlc_config &c = p.cfg;
  const Layout L = run_layout(p);
  rc = upload_index(p, ws, L, s);
  if (rc) return rc;
  if (tb.n_tri && p.n_tri > 0) {  // the workspace keeps the counts this run used
    rc = hip_check(hipMemcpyAsync(at<double>(ws, L, B_NTRI), tb.n_tri, (size_t)p.n_tri * 8, hipMemcpyDeviceToDevice,
                                  s), "triangle counts");
    if (rc) return rc;
  }
  const DevTables T = dev_tables(p, tb, rho);
  const double *cent = at<double>(ws, L, B_CENT);
  const int n_cfg = (int)p.cfgs.size();
  const int32_t *cfgT = at<int32_t>(ws, L, B_CFGT);
  const int32_t *rowR = at<int32_t>(ws, L, B_ROWR);
  double *U = at<double>(ws, L, B_U), *Pk = at<double>(ws, L, B_PK), *Ne = at<double>(ws, L, B_NE);
  double *X = at<double>(ws, L, B_X), *R = at<double>(ws, L, B_R);
  double *dR = at<double>(ws, L, B_DR), *rR = at<double>(ws, L, B_RR);
  double *Ps = at<double>(ws, L, B_PS);
  double *G = at<double>(ws, L, B_G), *Gmax = at<double>(ws, L, B_GMAX), *Ts = at<double>(ws, L, B_TS);
  int32_t *sexp = at<int32_t>(ws, L, B_SEXP);

  if (hooks) hooks->begin(WLC_PHASE_TABLES);
  const SubList sl{at<int32_t>(ws, L, B_SOFF), at<int32_t>(ws, L, B_SLEG), at<double>(ws, L, B_SWT)};
  launch_stage(T, cent, p.n_ell * p.n_sub, U, Pk, Ne, s);
  launch_spectra(T, cfgT, n_cfg, sl, U, Pk, Ne, cent, X, R, s);
  launch_project(T, rowR, cfgT, p.n_R, X, R, dR, rR, s);
  launch_ps(dR, Ps, p.n_ell, c.n_z, p.noise, s);
  const bool ssc_chi = (c.flags & WLC_FLAG_SSC_CHI) != 0;
  const int n_mg = g_cols(c);
  double *sw = ssc_chi ? at<double>(ws, L, B_SW) : nullptr;
  if (ssc_chi) launch_sigma_w2(T, theta_sky(p), sw, s);
  launch_gfactor(T, cfgT, n_cfg, sl, U, R, sw, std::sqrt(p.omega), n_mg, G, Gmax, s);
  launch_tfactor(T, rowR, cfgT, p.n_R, Gmax, Ts, sexp, s);
  const bool arows = !p.arow.empty();  // the flattened products run on A-rows in their own order
  const int32_t *arow = arows ? at<int32_t>(ws, L, B_AROW) : nullptr;
  const int32_t *pos = arows ? at<int32_t>(ws, L, B_POS) : nullptr;
  int32_t *ext = arows ? at<int32_t>(ws, L, B_EXT) : nullptr;
  if (arows) launch_panel_ext(Ts, arow, p.r_pad, c.n_chi, n_mg, p.k_pad, ext, s);
  if (c.precision == WLC_BF16_AUTO)
    launch_split_plan(asm_args(p, ws, L), rowR, Ts, G, p.n_R, n_cfg, c.n_chi, n_mg, at<double>(ws, L, B_SQ),
                      at<double>(ws, L, B_GD), at<double>(ws, L, B_FP), (int)(p.r_pad / GRAM_TILE), s, pos);
  if (c.flags & WLC_FLAG_NGINS) {
    // the projected one-halo trispectrum of two legs per triangle (the P.T
    // term), in FP64 through the factorisation along chi
    const int nz = c.n_z;
    double *Ts2 = at<double>(ws, L, B_TS2), *G2 = at<double>(ws, L, B_G2);
    launch_twoleg(T, p.n_ell, U, G2, Ts2, s);
    launch_chifact(Ts2, G2, at<double>(ws, L, B_H2), twoleg_configs(p), c.n_chi, c.n_m, p.n_ell,
                   nz * (nz + 1) / 2, nz * nz, twoleg_configs(p) - p.n_ell, at<double>(ws, L, B_T2), twoleg_ld(p), s);
  }
  if (hooks) hooks->end(WLC_PHASE_TABLES);

  // the flattened factor A (none in the chi-factorised form)
  if (hooks) hooks->begin(WLC_PHASE_ABUILD);
  if (c.precision != WLC_FP64_CHI) {
    const int fmt = c.precision == WLC_FP64 ? 0 : c.precision == WLC_BF16 ? 1 : c.precision == WLC_FP32 ? 3 : 2;
    const bool auto_split = c.precision == WLC_BF16_AUTO;
    launch_abuild(fmt, rowR, Ts, G, p.n_R, p.r_pad, c.n_chi, n_mg, p.k_pad, p.k_pad, at<void>(ws, L, B_A0),
                  at<void>(ws, L, B_A1), s, auto_split ? at<double>(ws, L, B_FP) : nullptr,
                  auto_split ? split_lim(p) : 0.0, arow, ext);
  }
  if (hooks) hooks->end(WLC_PHASE_ABUILD);
  return hip_check(hipGetLastError(), "run launch");
}

static GramShape gram_shape(const Plan &p) { return GramShape{p.r_pad, p.k_pad, p.r_pad, p.k_pad}; }

// WLC_BF16_AUTO: tile (I, J) takes the split product iff
// (2u + u^2 + K 2^-24) sqrt(F_I F_J) > tol, i.e. F_I F_J > lim, with
// u = 2^-8 (bf16 operands rounded to nearest) and K 2^-24 the FP32
// accumulation of K products.
static double split_lim(const Plan &p) {
  const double tol = p.cfg.gram_tol > 0.0 ? p.cfg.gram_tol : std::ldexp(1.0, -17);
  const double u = std::ldexp(1.0, -8);
  const double eps = 2.0 * u + u * u + (double)p.k_pad * std::ldexp(1.0, -24);
  return (tol / eps) * (tol / eps);
}

// The flattened product goes to GP (A-row order) and is put back in the
// distinct-row order by run_enqueue_back; the chi-factorised one writes G
// directly.
static void *gram_out(const Plan &p, void *ws, const Layout &L) {
  return at<void>(ws, L, p.arow.empty() ? B_GM : B_GP);
}
static const int32_t *gram_ext(const Plan &p, void *ws, const Layout &L) {
  return p.arow.empty() ? nullptr : at<int32_t>(ws, L, B_EXT);
}

int run_enqueue_gram(const Plan &p, void *ws, hipStream_t s, PhaseHooks *hooks) {
  const wlc_config &c = p.cfg;
  const Layout L = run_layout(p);
  void *Gm = gram_out(p, ws, L);
  if (hooks) hooks->begin(WLC_PHASE_GRAM);
  if (c.precision == WLC_FP64_CHI) {
    // no flattened factor: the one-halo product from T and G directly
    const int nz = c.n_z;
    launch_chifact(at<double>(ws, L, B_TS), at<double>(ws, L, B_G), at<double>(ws, L, B_H), (int)p.cfgs.size(),
                   c.n_chi, g_cols(c), p.n_ell, nz * (nz + 1) / 2, nz * (nz + 1) * (nz + 2) / 6, p.n_tri,
                   (double *)Gm, p.r_pad, s);
  } else {
    launch_gram(c.precision, gram_shape(p), at<void>(ws, L, B_A0), at<void>(ws, L, B_A1), Gm, at<void>(ws, L, B_PART),
                s, at<double>(ws, L, B_FP), split_lim(p), gram_ext(p, ws, L));
  }
  if (hooks) hooks->end(WLC_PHASE_GRAM);
  return hip_check(hipGetLastError(), "gram launch");
}

bool run_gram_batchable(const Plan &p) { return gram_batchable(p.cfg.precision); }

void run_gram_job(const Plan &p, void *ws, GramJob &job) {
  const Layout L = run_layout(p);
  gram_job(p.cfg.precision, gram_shape(p), at<void>(ws, L, B_A0), at<void>(ws, L, B_A1), gram_out(p, ws, L),
           at<void>(ws, L, B_PART), job, at<double>(ws, L, B_FP), split_lim(p), gram_ext(p, ws, L));
}

int run_enqueue_gram_reduce(const Plan &p, void *ws, hipStream_t s) {
  const Layout L = run_layout(p);
  launch_gram_reduce(p.cfg.precision, gram_shape(p), gram_out(p, ws, L), at<void>(ws, L, B_PART), s);
  return hip_check(hipGetLastError(), "gram reduce launch");
}

static AsmArgs asm_args(const Plan &p, void *ws, const Layout &L) {
  const wlc_config &c = p.cfg;
  const bool ssc_chi = (c.flags & WLC_FLAG_SSC_CHI) != 0;
  AsmArgs a{};
  a.rowO = at<int32_t>(ws, L, B_ROWO);
  a.cfgT = at<int32_t>(ws, L, B_CFGT);
  a.sexp = at<int32_t>(ws, L, B_SEXP);
  a.Gm = at<void>(ws, L, B_GM);
  a.ld_g = p.r_pad;
  a.gm_f32 = !prec_f64(c.precision);
  a.Ps = at<double>(ws, L, B_PS);
  a.nmodes = at<double>(ws, L, B_NMODES);
  a.ntri = at<double>(ws, L, B_NTRI);
  a.rR = at<double>(ws, L, B_RR);
  a.dR = at<double>(ws, L, B_DR);
  a.n_z = c.n_z;
  a.n_ell = p.n_ell;
  a.n = p.n_out;
  a.omega = p.omega;
  a.inv_omega = 1.0 / p.omega;
  a.sigma_b2 = ssc_chi ? 0.0 : c.sigma_b2;  // else inside the Gram product
  a.ngins = (c.flags & WLC_FLAG_NGINS) != 0;
  a.T2 = a.ngins ? at<double>(ws, L, B_T2) : nullptr;
  a.ld_t2 = a.ngins ? twoleg_ld(p) : 0;
  return a;
}

int run_enqueue_back(const Plan &p, const wlc_tables &tb, void *ws, double *d, double *r, void *C, int32_t *row_exp2,
                     hipStream_t s, PhaseHooks *hooks) {
  (void)tb;
  const wlc_config &c = p.cfg;
  const Layout L = run_layout(p);
  void *Gm = at<void>(ws, L, B_GM);
  const AsmArgs a = asm_args(p, ws, L);
  if (hooks) hooks->begin(WLC_PHASE_ASSEMBLE);
  if (p.arow.empty()) {
    launch_gram_mirror(a.gm_f32, Gm, p.n_R, p.r_pad, s);
  } else {  // the product of the A-rows, made symmetric, back in the distinct-row order
    void *GP = at<void>(ws, L, B_GP);
    launch_gram_mirror(a.gm_f32, GP, p.r_pad, p.r_pad, s);
    launch_gram_unpermute(a.gm_f32, GP, at<int32_t>(ws, L, B_POS), p.n_R, p.r_pad, Gm, s);
  }
  launch_rowexp(a, row_exp2, d, r, s);
  launch_assemble(a, row_exp2, C, s);
  if (hooks) hooks->end(WLC_PHASE_ASSEMBLE);
  return hip_check(hipGetLastError(), "run launch");
}

int run_enqueue(const Plan &p, const wlc_tables &tb, void *ws, double *d, double *r, void *C, int32_t *row_exp2,
                hipStream_t s, PhaseHooks *hooks, double rho) {
  int rc = run_enqueue_front(p, tb, ws, s, hooks, rho);
  if (!rc) rc = run_enqueue_gram(p, ws, s, hooks);
  if (!rc) rc = run_enqueue_back(p, tb, ws, d, r, C, row_exp2, s, hooks);
  return rc;
}

int snr_enqueue(const Plan &p, const void *C, const int32_t *row_exp2, const double *d, void *ws, hipStream_t s,
                PhaseHooks *hooks, KernelProbe *probe, int32_t **flag_dev, double **out_dev, bool lmax) {
  const int64_t n = p.n_out, ld = snr_ld(n);
  char *base = static_cast<char *>(ws);
  double *Wm = reinterpret_cast<double *>(base);
  size_t o = align_up((size_t)(n + 1) * ld * 8, 256);
  double *scratch = reinterpret_cast<double *>(base + o);
  o += align_up(chol_scratch_bytes(n), 256);
  int32_t *flag = reinterpret_cast<int32_t *>(base + o);
  o += 256;
  double *out = reinterpret_cast<double *>(base + o);
  o += 256;
  int32_t *perm = reinterpret_cast<int32_t *>(base + o);
  o += align_up((size_t)n * 4, 256);
  int32_t *ends = reinterpret_cast<int32_t *>(base + o);
  o += align_up((size_t)p.n_ell * 8, 256);
  double *part = reinterpret_cast<double *>(base + o);
  o += align_up((size_t)p.n_ell * 8, 256);
  double *curve = reinterpret_cast<double *>(base + o);
  if (lmax) {
    int rc = hip_check(hipMemcpyAsync(perm, p.lmax_perm.data(), (size_t)n * 4, hipMemcpyHostToDevice, s), "perm upload");
    if (!rc)
      rc = hip_check(hipMemcpyAsync(ends, p.lmax_ends.data(), (size_t)p.n_ell * 4, hipMemcpyHostToDevice, s),
                     "ends upload");
    if (rc) return rc;
  }
  if (hooks) hooks->begin(WLC_PHASE_SNR_PREP);
  launch_fill_i32(flag, 1, 0, s);
  launch_chol_prep(C, !prec_f64(p.cfg.precision), row_exp2, d, n, ld, Wm, s, lmax ? perm : nullptr);
  if (hooks) hooks->end(WLC_PHASE_SNR_PREP);
  if (hooks) hooks->begin(WLC_PHASE_CHOL);
  chol_factor(Wm, n, ld, scratch, flag, s, probe);
  if (lmax)
    launch_sumsq_groups(Wm, n, ld, ends, p.n_ell, part, curve, s);
  else
    launch_sumsq_row(Wm, n, ld, out, s);
  if (hooks) hooks->end(WLC_PHASE_CHOL);
  *flag_dev = flag;
  *out_dev = lmax ? curve : out;
  return hip_check(hipGetLastError(), "snr launch");
}

// ---- fixed device scratch of wlc_snr2_noalloc
// One array per device, holding the bordered matrix, the Cholesky's split-k
// partials, the pivot flag and the result of one S/N at a time.  Host code
// never uses the array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char snr_scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[MAX_DEVICES] = {};

static int noalloc_scratch(void **out) {
  int dev = 0;
  int rc = hip_check(hipGetDevice(&dev), "current device");
  if (rc) return rc;
  if (dev < 0 || dev >= MAX_DEVICES) return fail(WLC_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    rc = hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(snr_scratch)), "scratch address");
    if (rc) return rc;
    if (!ptr) return fail(WLC_EDEVICE, "scratch address is null");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return WLC_OK;
}

__global__ void k_copy_snr_result(const int32_t *flag, const double *out, int32_t *status, double *snr2) {
  if (threadIdx.x == 0) {
    status[0] = flag[0];
    snr2[0] = out[0];
  }
}

int snr_noalloc_enqueue(const Plan &p, const void *C, const int32_t *row_exp2, const double *d, double *snr2_dev,
                        int32_t *status_dev, hipStream_t s) {
  const size_t need = snr_ws_bytes(p);
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(WLC_EINVAL, "the data vector is too long for the fixed S/N scratch (" +
                                std::to_string(need >> 20) + " MiB needed, 64 MiB available)");
  void *ws = nullptr;
  int rc = noalloc_scratch(&ws);
  if (rc) return rc;
  int32_t *flag = nullptr;
  double *out = nullptr;
  rc = snr_enqueue(p, C, row_exp2, d, ws, s, nullptr, nullptr, &flag, &out);
  if (rc) return rc;
  hipLaunchKernelGGL(k_copy_snr_result, dim3(1), dim3(64), 0, s, flag, out, status_dev, snr2_dev);
  return hip_check(hipGetLastError(), "snr launch");
}

int plan_build(const wlc_config &cfg, Plan &p) {
  int rc = build_plan(cfg, p);
  if (rc) return rc;
  finish_sizes(p);
  return WLC_OK;
}

}  // namespace wlc

using namespace wlc;

extern "C" {

const char *wlc_last_error(void) { return last_error(); }

int wlc_plan_set_timing(wlc_plan plan, int enable) {
  if (!plan) return fail(WLC_EINVAL, "null plan");
  if (enable && !plan->events_ready) {
    for (auto &e : plan->ev) {
      int rc = hip_check(hipEventCreate(&e), "event create");
      if (rc) return rc;
    }
    // two events per block-update launch: about 5 launches per 256 columns
    const int64_t launches = 5 * ((plan->p.n_out + 255) / 256) + 16;
    plan->upd_ev.resize((size_t)std::min<int64_t>(2 * launches, 16384));
    for (auto &e : plan->upd_ev) {
      int rc = hip_check(hipEventCreate(&e), "event create");
      if (rc) return rc;
    }
    plan->events_ready = true;
  }
  plan->timing = enable != 0;
  return WLC_OK;
}

int wlc_plan_kernel_stats(wlc_plan plan, double *ms_total, int64_t *launches, int64_t *timed, double *flops) {
  if (!plan || !ms_total || !launches || !timed || !flops) return fail(WLC_EINVAL, "null argument");
  *ms_total = 0.0;
  *launches = 0;
  *timed = 0;
  *flops = 0.0;
  if (!plan->probe_valid) return WLC_OK;
  const KernelProbe &pr = plan->probe;
  for (int q = 0; q < pr.count; ++q) {
    float m = 0.0f;
    int rc = hip_check(hipEventSynchronize(pr.ev[2 * q + 1]), "event sync");
    if (!rc) rc = hip_check(hipEventElapsedTime(&m, pr.ev[2 * q], pr.ev[2 * q + 1]), "event time");
    if (rc) return rc;
    *ms_total += m;
  }
  *launches = pr.launches;
  *timed = pr.count;
  *flops = pr.flops;
  return WLC_OK;
}

int wlc_plan_timings(wlc_plan plan, float *ms) {
  if (!plan || !ms) return fail(WLC_EINVAL, "null argument");
  for (int ph = 0; ph < WLC_PHASE_COUNT; ++ph) {
    ms[ph] = 0.0f;
    if (!plan->events_ready || !plan->recorded[ph]) continue;
    int rc = hip_check(hipEventSynchronize(plan->ev[2 * ph + 1]), "event sync");
    if (!rc) rc = hip_check(hipEventElapsedTime(&ms[ph], plan->ev[2 * ph], plan->ev[2 * ph + 1]), "event time");
    if (rc) return rc;
  }
  return WLC_OK;
}

int wlc_plan_create(const wlc_config *cfg, wlc_plan *out) {
  if (!cfg || !out) return fail(WLC_EINVAL, "null argument");
  *out = nullptr;
  try {
    auto *h = new wlc_plan_s();
    int rc = plan_build(*cfg, h->p);
    if (rc) {
      delete h;
      return rc;
    }
    *out = h;
    return WLC_OK;
  } catch (const std::bad_alloc &) {
    return fail(WLC_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(WLC_EINVAL, "plan construction failed");
  }
}

void wlc_plan_destroy(wlc_plan plan) { delete plan; }

int wlc_plan_sizes(wlc_plan plan, wlc_sizes *out) {
  if (!plan || !out) return fail(WLC_EINVAL, "null argument");
  const Plan &p = plan->p;
  out->n_data = p.n_out;
  out->n_distinct = p.n_R;
  out->n_p = p.n_p;
  out->n_tri = p.n_tri;
  out->n_cfg = (int64_t)p.cfgs.size();
  out->n_ell_used = p.n_ell;
  out->k_len = p.k_len;
  out->c_elem_bytes = prec_f64(p.cfg.precision) ? 8 : 4;
  out->ws_run_bytes = p.ws_run;
  out->ws_snr_bytes = p.ws_snr;
  out->ws_snr_structured_bytes = snr_structured_ws_bytes(p);
  out->n_avg = (int64_t)p.sub_w.size();
  out->ws_pca_bytes = pca_ws_bytes(p);
  return WLC_OK;
}

int wlc_plan_averaging(wlc_plan plan, int32_t *off, int32_t *legs, double *ell, double *w) {
  if (!plan) return fail(WLC_EINVAL, "null plan");
  const Plan &p = plan->p;
  if (off) std::memcpy(off, p.sub_off.data(), p.sub_off.size() * 4);
  if (legs)
    for (size_t e = 0; e < p.sub_w.size(); ++e)
      for (int a = 0; a < 3; ++a) legs[3 * e + a] = p.sub_leg[4 * e + a];
  if (ell) std::memcpy(ell, p.sub_centres.data(), p.sub_centres.size() * 8);
  if (w) std::memcpy(w, p.sub_w.data(), p.sub_w.size() * 8);
  return WLC_OK;
}

int wlc_plan_index(wlc_plan plan, int32_t *tri, int32_t *rows, int32_t *distinct) {
  if (!plan) return fail(WLC_EINVAL, "null plan");
  const Plan &p = plan->p;
  if (tri)
    for (int t = 0; t < p.n_tri; ++t)
      for (int a = 0; a < 3; ++a) tri[3 * t + a] = p.cfgs[p.n_ell + t].leg[a];
  for (int64_t a = 0; a < p.n_out; ++a) {
    const int32_t *r = &p.rowO[8 * a];
    const int kind = p.cfgs[r[0]].kind;
    if (rows) {
      int32_t *o = rows + 8 * a;
      o[0] = kind;
      o[1] = r[0];
      o[2] = r[5]; o[3] = r[6]; o[4] = r[7];
      o[5] = r[2]; o[6] = r[3]; o[7] = r[4];
    }
    if (distinct) distinct[a] = r[1];
  }
  return WLC_OK;
}

int wlc_plan_gram_order(wlc_plan plan, int32_t *pos) {
  if (!plan || !pos) return fail(WLC_EINVAL, "null argument");
  const Plan &p = plan->p;
  for (int64_t e = 0; e < p.n_R; ++e) pos[e] = p.pos.empty() ? (int32_t)e : p.pos[(size_t)e];
  return WLC_OK;
}

int wlc_counts_closed(wlc_plan plan, double *n_modes, double *n_tri) {
  if (!plan) return fail(WLC_EINVAL, "null plan");
  const Plan &p = plan->p;
  if (n_modes) std::memcpy(n_modes, p.n_modes.data(), p.n_modes.size() * 8);
  if (n_tri) std::memcpy(n_tri, p.n_tri_closed.data(), p.n_tri_closed.size() * 8);
  return WLC_OK;
}

int wlc_lattice_counts(wlc_plan plan, void *ws, uint64_t *modes, uint64_t *tris, void *stream) {
  if (!plan || !ws) return fail(WLC_EINVAL, "null argument");
  const Plan &p = plan->p;
  hipStream_t s = (hipStream_t)stream;
  const Layout L = run_layout(p);
  // only the thresholds and the triangle legs: the workspace may hold the
  // triangle counts of a completed run, which a later structured S/N reads
  const Upload ups[] = {{B_THR, p.lattice_thr.data(), p.lattice_thr.size() * 8},
                        {B_TRI, p.triT.data(), p.triT.size() * 4}};
  int rc = upload(ups, 2, ws, L, s);
  if (rc) return rc;
  const int64_t thr_max = p.lattice_thr[p.n_ell];
  launch_lattice(at<int64_t>(ws, L, B_THR), thr_max, p.n_ell, at<int32_t>(ws, L, B_TRI), p.n_tri, modes, tris, s);
  return hip_check(hipGetLastError(), "lattice launch");
}

int wlc_run(wlc_plan plan, const wlc_tables *tb, void *ws, double *d, double *r, void *C, int32_t *row_exp2,
            void *stream) {
  if (!plan || !tb || !ws || !d || !r || !C || !row_exp2) return fail(WLC_EINVAL, "null argument");
  if (((uintptr_t)ws & 255) != 0) return fail(WLC_EINVAL, "workspace must be 256-byte aligned");
  const Plan &p = plan->p;
  hipStream_t s = (hipStream_t)stream;
  if (!(p.cfg.flags & WLC_FLAG_NOCHECK)) {
    int rc = validate_tables(p, *tb, ws, s);
    if (rc) return rc;
  }
  for (int ph = WLC_PHASE_TABLES; ph <= WLC_PHASE_ASSEMBLE; ++ph) plan->recorded[ph] = false;
  PlanTimer tm(plan, s);
  const bool timed = plan->timing && plan->events_ready;
  return run_enqueue(p, *tb, ws, d, r, C, row_exp2, s, timed ? &tm : nullptr);
}

int wlc_sigma_w2(wlc_plan plan, const wlc_tables *tb, double *sw, void *stream) {
  if (!plan || !tb || !sw || !tb->chi || !tb->k || !tb->P) return fail(WLC_EINVAL, "null argument");
  const Plan &p = plan->p;
  launch_sigma_w2(dev_tables(p, *tb), theta_sky(p), sw, (hipStream_t)stream);
  return hip_check(hipGetLastError(), "sigma_W^2 launch");
}

int wlc_snr2(wlc_plan plan, const void *C, const int32_t *row_exp2, const double *d, void *ws, double *snr2_host,
             void *stream) {
  if (!plan || !C || !row_exp2 || !d || !ws || !snr2_host) return fail(WLC_EINVAL, "null argument");
  if (((uintptr_t)ws & 255) != 0) return fail(WLC_EINVAL, "workspace must be 256-byte aligned");
  const Plan &p = plan->p;
  hipStream_t s = (hipStream_t)stream;
  plan->recorded[WLC_PHASE_SNR_PREP] = plan->recorded[WLC_PHASE_CHOL] = false;
  PlanTimer tm(plan, s);
  const bool timed = plan->timing && plan->events_ready;
  KernelProbe *probe = nullptr;
  if (timed) {
    plan->probe = KernelProbe{};
    plan->probe.ev = plan->upd_ev.data();
    plan->probe.cap = (int)plan->upd_ev.size() / 2;
    probe = &plan->probe;
    plan->probe_valid = true;
  }
  int32_t *flag = nullptr;
  double *out = nullptr;
  int rc = snr_enqueue(p, C, row_exp2, d, ws, s, timed ? &tm : nullptr, probe, &flag, &out);
  if (rc) return rc;
  struct { int32_t flag; int32_t pad; double v; } h{};
  rc = hip_check(hipMemcpyAsync(&h.flag, flag, 4, hipMemcpyDeviceToHost, s), "snr copy");
  if (!rc) rc = hip_check(hipMemcpyAsync(&h.v, out, 8, hipMemcpyDeviceToHost, s), "snr copy");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "snr sync");
  if (rc) return rc;
  if (h.flag) return fail(WLC_ENOTPD, "covariance is not positive definite");
  *snr2_host = h.v;
  return WLC_OK;
}

int wlc_gram_split_tiles(wlc_plan plan, const void *ws_run, int64_t *split, int64_t *tiles) {
  if (!plan || !ws_run || !split || !tiles) return fail(WLC_EINVAL, "null argument");
  const Plan &p = plan->p;
  const int64_t np = p.r_pad / GRAM_TILE;
  *tiles = p.cfg.precision == WLC_FP64_CHI ? 0 : np * (np + 1) / 2;
  *split = p.cfg.precision == WLC_BF16X3 ? *tiles : 0;
  if (p.cfg.precision != WLC_BF16_AUTO) return WLC_OK;
  const Layout L = run_layout(p);
  std::vector<double> F((size_t)np);
  int rc = hip_check(hipDeviceSynchronize(), "split plan sync");  // the run may be on any stream
  if (!rc)
    rc = hip_check(hipMemcpy(F.data(), static_cast<const char *>(ws_run) + L.off[B_FP], (size_t)np * 8,
                             hipMemcpyDeviceToHost), "split plan copy");
  if (rc) return rc;
  const double lim = split_lim(p);
  int64_t n = 0;
  for (int64_t I = 0; I < np; ++I)
    for (int64_t J = 0; J <= I; ++J) n += F[I] * F[J] > lim;
  *split = n;
  return WLC_OK;
}

// ---- the Gram product of a caller's factor (the kernels of wlc_run's one-halo term)
static int gram_shape_of(int precision, int64_t n, int64_t k, GramShape &g) {
  if (precision != WLC_BF16 && precision != WLC_BF16X3 && precision != WLC_BF16_AUTO)
    return fail(WLC_EINVAL, "wlc_gram: precision must be WLC_BF16, WLC_BF16X3 or WLC_BF16_AUTO");
  // the tile count and work items stay within the launch and int ranges
  if (n < 1 || k < 1 || n > ((int64_t)1 << 20) || k > ((int64_t)1 << 30))
    return fail(WLC_EINVAL, "wlc_gram: n or k out of range");
  const int64_t n_pad = round_up(n, GRAM_TILE), k_pad = round_up(k, 64);
  g = GramShape{n_pad, k_pad, n_pad, k_pad};
  return WLC_OK;
}

int wlc_gram_ws_bytes(int precision, int64_t n, int64_t k, size_t *bytes) {
  if (!bytes) return fail(WLC_EINVAL, "null argument");
  GramShape g;
  const int rc = gram_shape_of(precision, n, k, g);
  if (rc) return rc;
  *bytes = gram_partial_bytes(precision, g);
  return WLC_OK;
}

int wlc_gram(int precision, int64_t n, int64_t k, const uint16_t *a_hi, const uint16_t *a_lo,
             const double *panel_f, double lim, const int32_t *panel_ext, float *g, void *ws, void *stream) {
  GramShape sh;
  int rc = gram_shape_of(precision, n, k, sh);
  if (rc) return rc;
  if (!a_hi || !g) return fail(WLC_EINVAL, "wlc_gram: null A or G");
  if (precision != WLC_BF16 && !a_lo) return fail(WLC_EINVAL, "wlc_gram: the split products need a_lo");
  if (precision == WLC_BF16_AUTO && !panel_f) return fail(WLC_EINVAL, "wlc_gram: WLC_BF16_AUTO needs panel_f");
  const size_t part = gram_partial_bytes(precision, sh);
  if (part > 0 && !ws) return fail(WLC_EINVAL, "wlc_gram: null workspace");
  if (((uintptr_t)ws & 255) != 0) return fail(WLC_EINVAL, "wlc_gram: workspace must be 256-byte aligned");
  launch_gram(precision, sh, a_hi, precision == WLC_BF16 ? a_hi : a_lo, g, ws, (hipStream_t)stream,
              precision == WLC_BF16_AUTO ? panel_f : nullptr, precision == WLC_BF16_AUTO ? lim : 0.0, panel_ext);
  return hip_check(hipGetLastError(), "wlc_gram launch");
}

int wlc_gram_work(wlc_plan plan, const void *ws_run, double *flops, double *mfma_flops, double *factor_bytes) {
  if (!plan || !ws_run || !flops || !mfma_flops) return fail(WLC_EINVAL, "null argument");
  const Plan &p = plan->p;
  const int prec = p.cfg.precision;
  if (prec == WLC_FP64_CHI) {
    *flops = *mfma_flops = 0.0;
    if (factor_bytes) *factor_bytes = 0.0;
    return WLC_OK;
  }
  const Layout L = run_layout(p);
  int src = hip_check(hipDeviceSynchronize(), "gram work sync");  // the run may be on any stream
  if (src) return src;
  // 256-row panels: the units of the panel extents and of the per-tile precision
  const int64_t np = p.r_pad / GRAM_TILE;
  std::vector<int32_t> ext;
  if (!p.arow.empty()) {
    ext.resize((size_t)np);
    int rc = hip_check(hipMemcpy(ext.data(), static_cast<const char *>(ws_run) + L.off[B_EXT], (size_t)np * 4,
                                 hipMemcpyDeviceToHost), "panel extent copy");
    if (rc) return rc;
  }
  std::vector<double> F;
  if (prec == WLC_BF16_AUTO) {
    F.resize((size_t)np + 1);  // per panel, then the largest
    int rc = hip_check(hipMemcpy(F.data(), static_cast<const char *>(ws_run) + L.off[B_FP], (size_t)(np + 1) * 8,
                                 hipMemcpyDeviceToHost), "split plan copy");
    if (rc) return rc;
  }
  // k summed by a tile of panels I and J: up to the shorter extent, or all of K
  auto k_of = [&](int64_t I, int64_t J) {
    return ext.empty() ? (double)p.k_pad : (double)GRAM_KB * std::min(ext[(size_t)I], ext[(size_t)J]);
  };
  const double lim = split_lim(p);
  double f = 0.0, m = 0.0;
  if (prec == WLC_FP64 && gram_f64_tiles(gram_shape(p))) {
    // two 128 x 256 tiles (row halves of panel P) per panel pair P >= J
    for (int64_t P = 0; P < np; ++P)
      for (int64_t J = 0; J <= P; ++J) f += 2.0 * 2.0 * 128.0 * 256.0 * k_of(P, J);
    m = f;
  } else if (prec == WLC_FP64 || prec == WLC_FP32) {
    // 128 x 128 tiles over the lower triangle, in 256-row panels I / 2, J / 2
    const int64_t nt = p.r_pad / 128;
    for (int64_t I = 0; I < nt; ++I)
      for (int64_t J = 0; J <= I; ++J) f += 2.0 * 128.0 * 128.0 * k_of(I / 2, J / 2);
    m = f;
  } else {
    const double t2 = 2.0 * (double)GRAM_TILE * (double)GRAM_TILE;
    for (int64_t I = 0; I < np; ++I)
      for (int64_t J = 0; J <= I; ++J) {
        const double one = t2 * k_of(I, J);
        f += one;
        const bool split = prec == WLC_BF16X3 || (prec == WLC_BF16_AUTO && F[(size_t)I] * F[(size_t)J] > lim);
        m += split ? 3.0 * one : one;
      }
  }
  *flops = f;
  *mfma_flops = m;
  if (factor_bytes) {
    double b = 0.0;
    if (ext.empty() || prec == WLC_FP64) {  // the FP64 factor is written over all of K
      b = (double)p.n_R * (double)p.k_len * (prec == WLC_FP64 ? 8.0 : prec == WLC_FP32 ? 4.0 : 2.0);
    } else {  // the distinct rows lead the A-row order; a panel's rows end at its extent
      for (int64_t P = 0; P < np; ++P) {
        const int64_t tile = GRAM_TILE;
        const double rows = (double)std::max<int64_t>(0, std::min<int64_t>(tile, p.n_R - P * tile));
        const double k = (double)std::min<int64_t>((int64_t)GRAM_KB * ext[(size_t)P], p.k_len);
        const bool lo = prec == WLC_BF16X3 || (prec == WLC_BF16_AUTO && F[(size_t)P] * F[(size_t)np] > lim);
        b += rows * k * (lo ? 4.0 : 2.0);
      }
    }
    *factor_bytes = b;
  }
  return WLC_OK;
}

int wlc_snr2_noalloc(wlc_plan plan, const void *C, const int32_t *row_exp2, const double *d, double *snr2_dev,
                     int32_t *status_dev, void *stream) {
  if (!plan || !C || !row_exp2 || !d || !snr2_dev || !status_dev) return fail(WLC_EINVAL, "null argument");
  return snr_noalloc_enqueue(plan->p, C, row_exp2, d, snr2_dev, status_dev, (hipStream_t)stream);
}

int wlc_snr2_lmax(wlc_plan plan, const void *C, const int32_t *row_exp2, const double *d, void *ws,
                  double *snr2_host, void *stream) {
  if (!plan || !C || !row_exp2 || !d || !ws || !snr2_host) return fail(WLC_EINVAL, "null argument");
  if (((uintptr_t)ws & 255) != 0) return fail(WLC_EINVAL, "workspace must be 256-byte aligned");
  const Plan &p = plan->p;
  hipStream_t s = (hipStream_t)stream;
  plan->recorded[WLC_PHASE_SNR_PREP] = plan->recorded[WLC_PHASE_CHOL] = false;
  PlanTimer tm(plan, s);
  const bool timed = plan->timing && plan->events_ready;
  int32_t *flag = nullptr;
  double *out = nullptr;
  int rc = snr_enqueue(p, C, row_exp2, d, ws, s, timed ? &tm : nullptr, nullptr, &flag, &out, true);
  if (rc) return rc;
  int32_t hflag = 0;
  rc = hip_check(hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s), "snr copy");
  if (!rc) rc = hip_check(hipMemcpyAsync(snr2_host, out, (size_t)p.n_ell * 8, hipMemcpyDeviceToHost, s), "snr copy");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "snr sync");
  if (rc) return rc;
  if (hflag) return fail(WLC_ENOTPD, "covariance is not positive definite");
  return WLC_OK;
}

int wlc_pca(wlc_plan plan, const void *C, const int32_t *row_exp2, const double *d, void *ws, double *lambda,
            double *snr2_mode, double *cum_desc, int32_t *sweeps, double *S, void *stream) {
  if (!plan || !C || !row_exp2 || !d || !ws || !lambda || !snr2_mode || !cum_desc)
    return fail(WLC_EINVAL, "null argument");
  if (((uintptr_t)ws & 255) != 0) return fail(WLC_EINVAL, "workspace must be 256-byte aligned");
  const Plan &p = plan->p;
  if (pca_ws_bytes(p) == 0) return fail(WLC_EINVAL, "the PCA supports at most 65472 data-vector rows");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = p.n_out, np = pca_pad(p), ld = snr_ld(n);
  char *base = static_cast<char *>(ws);
  size_t o = align_up(snr_ws_bytes(p), 256);
  auto take = [&](size_t bytes) {
    char *q = base + o;
    o += align_up(bytes, 256);
    return q;
  };
  double *X = reinterpret_cast<double *>(take((size_t)np * np * 8));
  double *V = reinterpret_cast<double *>(take((size_t)np * np * 8));
  double *y = reinterpret_cast<double *>(take((size_t)np * 8));
  double *lam = reinterpret_cast<double *>(take((size_t)n * 8));
  double *snr = reinterpret_cast<double *>(take((size_t)n * 8));
  double *lam_out = reinterpret_cast<double *>(take((size_t)n * 8));
  double *snr_out = reinterpret_cast<double *>(take((size_t)n * 8));
  double *desc = reinterpret_cast<double *>(take((size_t)n * 8));
  int32_t *rank_lam = reinterpret_cast<int32_t *>(take((size_t)n * 4));
  int32_t *rank_snr = reinterpret_cast<int32_t *>(take((size_t)n * 4));
  double *conv = reinterpret_cast<double *>(take(256));
  const size_t pairs = (size_t)np / 64;
  double *part = reinterpret_cast<double *>(take(pairs * pca_slices(np) * 64 * 64 * 8));
  double *Qg = reinterpret_cast<double *>(take(pairs * 64 * 64 * 8));
  int32_t *rot = reinterpret_cast<int32_t *>(take(pairs * 4));
  // the bordered Cholesky: L of the scaled C and y = L^-1 2^t d
  int32_t *flag = nullptr;
  double *unused = nullptr;
  int rc = snr_enqueue(p, C, row_exp2, d, ws, s, nullptr, nullptr, &flag, &unused);
  if (rc) return rc;
  int32_t hflag = 0;
  rc = hip_check(hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s), "pca copy");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "pca sync");
  if (rc) return rc;
  if (hflag) return fail(WLC_ENOTPD, "covariance is not positive definite");
  double *Vr = S ? V : nullptr;
  launch_pca_init(reinterpret_cast<const double *>(ws), ld, row_exp2, n, np, X, Vr, y, s);
  const double tol = 8.0 * std::sqrt((double)np) * 2.220446049250313e-16;
  const int n_blk = (int)(np / 32);
  int used = 0;
  bool converged = false;
  for (int sweep = 0; sweep < 40 && !converged; ++sweep) {
    launch_fill_i32(reinterpret_cast<int32_t *>(conv), 2, 0, s);
    for (int r = 0; r < n_blk - 1; ++r) launch_pca_round(X, Vr, np, r, tol, PCA_INNER, conv, part, Qg, rot, s);
    double hconv = 0.0;
    rc = hip_check(hipMemcpyAsync(&hconv, conv, 8, hipMemcpyDeviceToHost, s), "pca copy");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "pca sync");
    if (rc) return rc;
    used = sweep + 1;
    converged = !(hconv > tol);
  }
  if (sweeps) *sweeps = used;
  if (!converged) return fail(WLC_ENOCONV, "the PCA Jacobi sweeps did not converge");
  launch_pca_finish(X, y, Vr, n, np, lam, snr, rank_lam, rank_snr, lam_out, snr_out, desc, S, s);
  rc = hip_check(hipMemcpyAsync(lambda, lam_out, (size_t)n * 8, hipMemcpyDeviceToHost, s), "pca copy");
  if (!rc) rc = hip_check(hipMemcpyAsync(snr2_mode, snr_out, (size_t)n * 8, hipMemcpyDeviceToHost, s), "pca copy");
  if (!rc) rc = hip_check(hipMemcpyAsync(cum_desc, desc, (size_t)n * 8, hipMemcpyDeviceToHost, s), "pca copy");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "pca sync");
  return rc;
}

int wlc_snr2_structured(wlc_plan plan, const void *ws_run, void *ws, double *snr2_host, void *stream) {
  if (!plan || !ws_run || !ws || !snr2_host) return fail(WLC_EINVAL, "null argument");
  if (((uintptr_t)ws & 255) != 0 || ((uintptr_t)ws_run & 255) != 0)
    return fail(WLC_EINVAL, "workspaces must be 256-byte aligned");
  const Plan &p = plan->p;
  hipStream_t s = (hipStream_t)stream;
  plan->recorded[WLC_PHASE_SNR_PREP] = plan->recorded[WLC_PHASE_CHOL] = false;
  PlanTimer tm(plan, s);
  const bool timed = plan->timing && plan->events_ready;
  KernelProbe *probe = nullptr;
  if (timed) {
    plan->probe = KernelProbe{};
    plan->probe.ev = plan->upd_ev.data();
    plan->probe.cap = (int)plan->upd_ev.size() / 2;
    probe = &plan->probe;
    plan->probe_valid = true;
  }
  int32_t *flag = nullptr;
  double *out = nullptr;
  int rc = snr_structured_enqueue(p, ws_run, ws, s, timed ? &tm : nullptr, probe, &flag, &out);
  if (rc) return rc;
  struct { int32_t flag; int32_t pad; double v; } h{};
  rc = hip_check(hipMemcpyAsync(&h.flag, flag, 4, hipMemcpyDeviceToHost, s), "snr copy");
  if (!rc) rc = hip_check(hipMemcpyAsync(&h.v, out, 8, hipMemcpyDeviceToHost, s), "snr copy");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "snr sync");
  if (rc) return rc;
  if (h.flag) return fail(WLC_ENOTPD, "covariance is not positive definite");
  *snr2_host = h.v;
  return WLC_OK;
}

}  // extern "C"
