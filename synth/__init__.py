"""Seeded synthetic input tables for the weak-lensing covariance path.

This module builds the *inputs* of the method -- lensing kernels W_i(chi),
linear power P(k, chi), halo mass function n(M), halo profile u(k, M) and the
chi / k / M grids with their quadrature weights -- from closed-form recipes.
It contains none of the method's own arithmetic (no halo integrals, no
projection, no covariance); both the HIP library and the CPU oracle consume
what it returns, and neither is imported here.

Recipes (the paper's inputs are analytic functions of a calibrated halo
model that is not reproduced; these stand in for them):

* flat LCDM background, c = 1, lengths in Mpc/h: chi(z) = int dz / H(z),
  H(z) = H0 sqrt(Om (1+z)^3 + 1 - Om), H0 = 1/2997.92458 h/Mpc
  (the background of Sec. 2 of the paper);
* sources n(z) ~ (z/z0)^2 exp(-(z/z0)^1.5) on [0.001, 2.5], z0 = 0.64, split
  in equipopulated bins (the Euclid-like survey of App. A);
* lensing kernel W_i(chi) = int dz_s n_i(z_s) (3/2) Om H0^2 (1+z) chi
  (chi_s - chi)/chi_s (eqs. KernelLensing1 and LensEff);
* P(k, chi) = A k / (1 + (k/0.02)^2)^1.4 * D(chi)^2 with A fixed by
  sigma_8 (top-hat, R = 8 Mpc/h) and D the LCDM growth factor, D(0) = 1;
* n(M) ~ M^-1.9 exp(-M/1e14) on log-spaced masses in [1e11, 1e16],
  normalised so that sum_m w_m (M_m/rho) n_m = 1 (the beta = 0 case of the
  mass-consistency relation, eq. BoundinMass);
* u(k, M) = exp(-(k r)^2 / 2), r = (3 M / (4 pi 200 rho))^(1/3), floored at
  1e-300 so that every table entry is strictly positive;
* chi nodes are the midpoints of [0, chi(2.5)] (weight = spacing), masses
  use the trapezoid rule in ln M, k is log-spaced from
  min(ell_min / (2 chi_max), 0.02 / (chi_max Theta)) to k_max, Theta the
  survey's angular radius (4 pi f_sky = 2 pi (1 - cos Theta)), so that
  the table also covers the variance of the long mode in the survey window
  (eps chi Theta <= 0.02 at the low end for every chi).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

H0 = 1.0 / 2997.92458          # h/Mpc with c = 1
RHO_CRIT = 2.775e11            # (M_sun/h) / (Mpc/h)^3
ARCMIN2_PER_SR = (10800.0 / math.pi) ** 2

# ---------------------------------------------------------------- presets
# Workload shapes.  "tiny": the small instance a CPU finishes in seconds;
# "euclid5": 5 equipopulated bins, 10 ell-bins over 20-3000, 256 x 128;
# "large10": 10 bins, 15 ell-bins over 10-5000, 512 x 256 (K = 131072).
PRESETS = {
    "tiny":    dict(n_z=2, n_ell=5, ell_min=100.0, ell_max=1000.0, n_chi=64, n_m=32, n_k=768),
    "mid":     dict(n_z=3, n_ell=7, ell_min=50.0, ell_max=2000.0, n_chi=96, n_m=48, n_k=768),
    "euclid5": dict(n_z=5, n_ell=10, ell_min=20.0, ell_max=3000.0, n_chi=256, n_m=128, n_k=768),
    "large10": dict(n_z=10, n_ell=15, ell_min=10.0, ell_max=5000.0, n_chi=512, n_m=256, n_k=768),
    # the paper's own binning (14 log ell-bins over 10-5000, App. A) on the
    # Euclid-like grid; n_z is chosen per use (1, 2 and 5 in its PCA study)
    "paper14": dict(n_z=5, n_ell=14, ell_min=10.0, ell_max=5000.0, n_chi=256, n_m=128, n_k=768),
}

SURVEY_DEFAULTS = dict(f_sky=0.36, sigma_eps=0.3, n_gal_arcmin2=30.0,
                       sigma_b2=1e-4, k_max=50.0)


@dataclasses.dataclass
class Tables:
    """Everything a run needs: scalar configuration plus float64 tables."""
    cfg: dict                 # n_z, n_ell, ell_min, ell_max, n_chi, n_m, n_k, survey scalars, rho_mean
    chi: np.ndarray           # [n_chi]
    w_chi: np.ndarray         # [n_chi]
    k: np.ndarray             # [n_k]
    m: np.ndarray             # [n_m]
    w_m: np.ndarray           # [n_m]
    W: np.ndarray             # [n_z][n_chi]
    P: np.ndarray             # [n_chi][n_k]
    u: np.ndarray             # [n_m][n_k]
    n_m: np.ndarray           # [n_m]
    b1: np.ndarray | None = None   # [n_m] or None (=> 1)
    b2: np.ndarray | None = None   # [n_m] or None (=> 0)
    z_edges: np.ndarray | None = None

    def arrays(self):
        return dict(chi=self.chi, w_chi=self.w_chi, k=self.k, m=self.m, w_m=self.w_m,
                    W=self.W, P=self.P, u=self.u, n_m=self.n_m, b1=self.b1, b2=self.b2)


# ---------------------------------------------------------- background
def _hubble(z, om):
    return H0 * np.sqrt(om * (1.0 + z) ** 3 + 1.0 - om)


def _cumtrapz(y, x):
    out = np.zeros_like(y)
    out[1:] = np.cumsum(0.5 * (y[1:] + y[:-1]) * np.diff(x))
    return out


def comoving_distance_table(om, z_max=2.5, n=20001):
    z = np.linspace(0.0, z_max, n)
    chi = _cumtrapz(1.0 / _hubble(z, om), z)
    return z, chi


def growth_table(om, z):
    """LCDM linear growth D(z)/D(0), D ~ H(a) int_0^a da' / (a' H(a'))^3."""
    a_grid = np.linspace(1e-6, 1.0, 200001)
    e = np.sqrt(om / a_grid ** 3 + 1.0 - om)
    integrand = 1.0 / (a_grid * e) ** 3
    cum = _cumtrapz(integrand, a_grid)
    d_of_a = e * cum
    d_of_a /= d_of_a[-1]
    a = 1.0 / (1.0 + z)
    return np.interp(a, a_grid, d_of_a)


# ---------------------------------------------------------- sources
def nz_shape(z, z0=0.64):
    return (z / z0) ** 2 * np.exp(-((z / z0) ** 1.5))


_EDGES = {}


def equipopulated_edges(n_bins, z0=0.64, z_min=0.001, z_max=2.5, n=200001):
    key = (int(n_bins), z0, z_min, z_max, n)
    if key not in _EDGES:
        z = np.linspace(z_min, z_max, n)
        cdf = _cumtrapz(nz_shape(z, z0), z)
        cdf /= cdf[-1]
        edges = np.interp(np.arange(1, n_bins) / n_bins, cdf, z)
        _EDGES[key] = np.concatenate([[z_min], edges, [z_max]])
    return _EDGES[key].copy()


def lensing_kernels(chi_nodes, om, z_edges, z0=0.64, nzs=6001):
    """W_i(chi) on the given chi nodes; each n_i has unit integral in its bin.

    The source integral int dz_s n_i(z_s) (chi_s - chi)/chi_s over chi_s > chi
    is the trapezoid rule on nzs nodes per bin, with the integrand set to 0
    at nodes where chi_s <= chi.  On a node grid sorted by chi_s it is the
    suffix sum over the segments above the crossing of
    0.5 dz (y_l + y_l+1), y = n_i - chi n_i/chi_s, plus the one segment
    through the crossing, whose lower node contributes 0."""
    chi_nodes = np.asarray(chi_nodes, np.float64)
    zt, chit = comoving_distance_table(om, z_max=max(2.5, z_edges[-1]), n=40001)
    z_of_chi = np.interp(chi_nodes, chit, zt)
    n_z = len(z_edges) - 1
    W = np.zeros((n_z, len(chi_nodes)))
    for i in range(n_z):
        zs = np.linspace(z_edges[i], z_edges[i + 1], nzs)
        ni = nz_shape(zs, z0)
        ni /= _cumtrapz(ni, zs)[-1]
        chis = np.interp(zs, zt, chit)
        dz = np.diff(zs)
        a = ni
        b = ni / np.where(chis > 0, chis, 1.0)
        # suffix sums of whole segments l .. nzs-2: S[l] = sum_{m >= l} 0.5 dz_m (f_m + f_m+1)
        seg_a = 0.5 * dz * (a[1:] + a[:-1])
        seg_b = 0.5 * dz * (b[1:] + b[:-1])
        Sa = np.concatenate([np.cumsum(seg_a[::-1])[::-1], [0.0]])
        Sb = np.concatenate([np.cumsum(seg_b[::-1])[::-1], [0.0]])
        # first node with chi_s > chi (chis increases with z_s)
        j = np.searchsorted(chis, chi_nodes, side="right")
        inside = j < nzs
        jj = np.minimum(j, nzs - 1)
        whole = Sa[jj] - chi_nodes * Sb[jj]            # segments entirely above the crossing
        part = np.where(j > 0, 0.5 * dz[np.maximum(jj - 1, 0)] * (a[jj] - chi_nodes * b[jj]), 0.0)
        # no node above the crossing: the bin lies entirely in front of chi
        integral = np.where(inside, whole + part, 0.0)
        # the chi node in front of the whole bin: every segment counts
        integral = np.where(j == 0, Sa[0] - chi_nodes * Sb[0], integral)
        W[i] = 1.5 * om * H0 ** 2 * (1.0 + z_of_chi) * chi_nodes * integral
    return W


# ---------------------------------------------------------- power spectrum
def plin_shape(k):
    return k / (1.0 + (k / 0.02) ** 2) ** 1.4


def sigma8_amplitude(sigma8=0.8, R=8.0):
    lk = np.linspace(math.log(1e-5), math.log(1e3), 400001)
    k = np.exp(lk)
    x = k * R
    wth = 3.0 * (np.sin(x) - x * np.cos(x)) / x ** 3
    small = x < 1e-3
    wth[small] = 1.0 - x[small] ** 2 / 10.0
    integrand = k ** 3 * plin_shape(k) * wth ** 2 / (2.0 * math.pi ** 2)
    s2 = _cumtrapz(integrand, lk)[-1]
    return sigma8 ** 2 / s2


# ---------------------------------------------------------- builder
def make_tables(preset="tiny", omega_m=0.3, sigma8=0.8, chi_grid_om=None,
                n_z=None, ell_cut=None, **overrides) -> Tables:
    """Build the synthetic tables for a preset shape.

    ``chi_grid_om`` fixes the chi grid to chi(2.5) of another Omega_m (the
    grid is shared by requests with different cosmologies); kernels vanish
    beyond each cosmology's own chi(2.5).
    """
    cfg = dict(PRESETS[preset]) if isinstance(preset, str) else dict(preset)
    cfg.update(SURVEY_DEFAULTS)
    if n_z is not None:
        cfg["n_z"] = n_z
    cfg.update(overrides)
    om = omega_m
    rho = om * RHO_CRIT
    cfg["rho_mean"] = rho
    cfg["omega_m"] = om
    cfg["sigma8"] = sigma8
    cfg["ell_cut"] = float(ell_cut) if ell_cut else 0.0

    zt, chit = comoving_distance_table(chi_grid_om if chi_grid_om else om)
    chi_max = chit[-1]
    n_chi = cfg["n_chi"]
    dchi = chi_max / n_chi
    chi = (np.arange(n_chi) + 0.5) * dchi
    w_chi = np.full(n_chi, dchi)

    z_edges = equipopulated_edges(cfg["n_z"])
    W = lensing_kernels(chi, om, z_edges)

    # k grid: from half the smallest ell over chi_max (or lower, down to the
    # scale of the survey window at chi_max) up to k_max
    n_k = cfg["n_k"]
    theta = math.acos(1.0 - 2.0 * cfg["f_sky"])
    k_lo = min(0.5 * cfg["ell_min"] / chi_max, 0.02 / (chi_max * theta))
    k = np.exp(np.linspace(math.log(k_lo), math.log(cfg["k_max"]), n_k))
    zt_om, chit_om = comoving_distance_table(om, n=40001)
    z_nodes = np.interp(chi, chit_om, zt_om, right=zt_om[-1])
    D = growth_table(om, z_nodes)
    A = sigma8_amplitude(sigma8)
    P = A * plin_shape(k)[None, :] * (D ** 2)[:, None]

    n_m_pts = cfg["n_m"]
    lnm = np.linspace(math.log(1e11), math.log(1e16), n_m_pts)
    m = np.exp(lnm)
    dln = lnm[1] - lnm[0]
    w_m = m * dln
    w_m[0] *= 0.5
    w_m[-1] *= 0.5
    nm = m ** -1.9 * np.exp(-m / 1e14)
    nm /= np.sum(w_m * (m / rho) * nm)
    r = (3.0 * m / (4.0 * math.pi * 200.0 * rho)) ** (1.0 / 3.0)
    u = np.exp(-0.5 * (k[None, :] * r[:, None]) ** 2)
    u = np.maximum(u, 1e-300)

    return Tables(cfg=cfg, chi=chi, w_chi=w_chi, k=k, m=m, w_m=w_m, W=W, P=P, u=u,
                  n_m=nm, z_edges=z_edges)


def with_bias(t: Tables) -> Tables:
    """The same tables with mass-dependent halo biases b1(M), b2(M).

    b1 has the shape 0.7 + (M / 1e13)^0.45, normalised so that
    sum_m w_m (M_m/rho) n_m b1_m = 1 (the beta = 1 case of the
    mass-consistency relation, eq. BoundinMass); b2 follows the published
    quadratic-bias fit of Lazeyras et al. (2016),
    b2 = 0.412 - 2.143 b1 + 0.929 b1^2 + 0.008 b1^3, which is negative for
    low-mass haloes and positive for massive ones."""
    rho = t.cfg["rho_mean"]
    shape = 0.7 + (t.m / 1e13) ** 0.45
    b1 = shape / np.sum(t.w_m * (t.m / rho) * t.n_m * shape)
    b2 = 0.412 - 2.143 * b1 + 0.929 * b1 ** 2 + 0.008 * b1 ** 3
    return dataclasses.replace(t, b1=b1, b2=b2)


def power_law_tables(n_z=2, n_ell=4, ell_min=100.0, ell_max=1000.0, n_chi=32, n_m=8,
                     n_k=256, alpha=-1.5, amp=1e4, w_const=1e-3, chi_max=3000.0):
    """Degenerate inputs with closed-form answers: P = amp k^alpha at every chi,
    constant kernels, u = 1 and a single effective mass scale."""
    cfg = dict(n_z=n_z, n_ell=n_ell, ell_min=ell_min, ell_max=ell_max, n_chi=n_chi,
               n_m=n_m, n_k=n_k, **SURVEY_DEFAULTS)
    cfg["k_max"] = 1e6
    cfg["rho_mean"] = 0.3 * RHO_CRIT
    cfg["ell_cut"] = 0.0
    dchi = chi_max / n_chi
    chi = (np.arange(n_chi) + 0.5) * dchi
    w_chi = np.full(n_chi, dchi)
    k = np.exp(np.linspace(math.log(0.5 * ell_min / chi_max), math.log(2.0 * ell_max / chi[0]), n_k))
    P = np.tile(amp * k ** alpha, (n_chi, 1))
    m = np.exp(np.linspace(math.log(1e12), math.log(1e14), n_m))
    w_m = np.full(n_m, 1.0 / n_m) * m
    nm = np.ones(n_m)
    nm /= np.sum(w_m * (m / cfg["rho_mean"]) * nm)
    u = np.ones((n_m, n_k))
    W = np.full((n_z, n_chi), w_const)
    return Tables(cfg=cfg, chi=chi, w_chi=w_chi, k=k, m=m, w_m=w_m, W=W, P=P, u=u, n_m=nm)


def sample_pairs(n, count, seed=42):
    """Seeded (a, b) pairs with a >= b for sampled covariance checks."""
    rng = np.random.default_rng(seed)
    a = rng.integers(0, n, size=count)
    b = rng.integers(0, n, size=count)
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    return np.stack([hi, lo], axis=1).astype(np.int64)


# ---------------------------------------------------------- serving stream
SERVE_GRID_OM = 0.28       # chi grid: midpoints of [0, chi(2.5; Omega_m = 0.28)]
SERVE_FID = dict(omega_m=0.3, sigma8=0.8)
PRESETS["serve"] = dict(n_z=10, n_ell=15, ell_min=10.0, ell_max=5000.0, n_chi=256, n_m=128, n_k=768)


def serving_fiducial() -> Tables:
    """Fiducial device-resident tables of the serving workload: the 15 ell-bins
    over 10-5000, 256 x 128 (chi, M) grid shared by every request."""
    return make_tables("serve", chi_grid_om=SERVE_GRID_OM, **SERVE_FID)


def serving_requests(n, seed=1234, qps=1.0, fid: Tables | None = None):
    """A seeded Poisson stream of likelihood-style requests.  Each draws
    Omega_m ~ U[0.28, 0.32], sigma_8 ~ U[0.78, 0.86], n_z in {3, 5, 7, 10} and
    l_max in {1000, 3000, 5000}; it rescales P by (sigma_8/0.8)^2 and n(M) by
    Omega_m/0.3 (with rho = Omega_m rho_crit) and carries its own lensing
    kernels on the shared chi grid.  Arrival times are exponential gaps at
    rate qps."""
    fid = fid or serving_fiducial()
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(n):
        om = float(rng.uniform(0.28, 0.32))
        s8 = float(rng.uniform(0.78, 0.86))
        nz = int(rng.choice([3, 5, 7, 10]))
        lmax = float(rng.choice([1000.0, 3000.0, 5000.0]))
        t += float(rng.exponential(1.0 / qps))
        W = lensing_kernels(fid.chi, om, equipopulated_edges(nz))
        out.append(dict(t_arrival=t, omega_m=om, sigma8=s8, n_z=nz, ell_max=lmax, W=W,
                        p_scale=(s8 / SERVE_FID["sigma8"]) ** 2, n_scale=om / SERVE_FID["omega_m"],
                        rho_mean=om * RHO_CRIT))
    return out


def request_tables(fid: Tables, req: dict) -> Tables:
    """The complete tables of one request (fiducial tables rescaled), for
    running it alone or through the oracle."""
    cfg = dict(fid.cfg)
    cfg["n_z"] = req["n_z"]
    cfg["rho_mean"] = req["rho_mean"]
    cfg["ell_cut"] = req["ell_max"]
    return Tables(cfg=cfg, chi=fid.chi, w_chi=fid.w_chi, k=fid.k, m=fid.m, w_m=fid.w_m, W=req["W"],
                  P=fid.P * req["p_scale"], u=fid.u, n_m=fid.n_m * req["n_scale"])
