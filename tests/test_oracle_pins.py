"""Pins of the FP64 oracle against values the paper prints, closed forms,
invariants and brute force.  CPU only."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ------------------------------------------------------------------ sizes
def _sizes(n_z, n_ell=14, lo=10.0, hi=5000.0, tomo="paper"):
    _, cen, _ = oracle.ell_bins(lo, hi, n_ell)
    rows = oracle.enumerate_rows(n_z, n_ell, cen, tomo)
    n_p = int(np.sum(rows["kind"] == 2))
    n_b = int(np.sum(rows["kind"] == 3))
    return n_p, n_b, rows


def test_paper_vector_sizes():
    g = _gold("paper_sizes.json")
    for nz, want in g["power_spectrum"].items():
        assert _sizes(int(nz))[0] == want
    for nz, want in g["bispectrum"].items():
        assert _sizes(int(nz))[1] == want
    for nz, want in g["joint"].items():
        p, b, _ = _sizes(int(nz))
        assert p + b == want


def test_triangle_classes_one_bin():
    _, cen, _ = oracle.ell_bins(10.0, 5000.0, 14)
    tris = oracle.triangles(cen)
    cls = [t[3] for t in tris]
    assert (len(tris), cls.count("E"), cls.count("I"), cls.count("S")) == (130, 14, 104, 12)
    # data-vector order: k slowest, then i, then j fastest
    keys = [(k, i, j) for (i, j, k, _) in tris]
    assert keys == sorted(keys)


@pytest.mark.parametrize("preset,n,n_p,n_tri,cls,n_sorted", [
    ("tiny", 143, 15, 22, (5, 14, 3), 103),
    ("euclid5", 4550, 150, 64, (10, 54, 0), 2390),
    ("large10", 82575, 825, 147, (15, 119, 13), 33165),
])
def test_workload_sizes(preset, n, n_p, n_tri, cls, n_sorted):
    p = synth.PRESETS[preset]
    _, cen, _ = oracle.ell_bins(p["ell_min"], p["ell_max"], p["n_ell"])
    rows = oracle.enumerate_rows(p["n_z"], p["n_ell"], cen)
    assert len(rows["kind"]) == n
    assert int(np.sum(rows["kind"] == 2)) == n_p
    tris = rows["triangles"]
    c = [t[3] for t in tris]
    assert len(tris) == n_tri and (c.count("E"), c.count("I"), c.count("S")) == cls
    srt = oracle.enumerate_rows(p["n_z"], p["n_ell"], cen, "sorted")
    assert len(srt["kind"]) == n_sorted
    canon, reps = oracle.canonical_rows(rows)
    assert len(reps) == n_sorted


def test_ell_edges_match_paper():
    g = _gold("paper_binning.json")
    edges, cen, wid = oracle.ell_bins(10.0, 5000.0, 14)
    assert np.max(np.abs(np.array(edges) - np.array(g["ell_edges_approx"]))) < 1.0
    # the bin is symmetric about its centre
    for e0, e1, c, w in zip(edges[:-1], edges[1:], cen, wid):
        assert abs(c - w / 2 - e0) < 1e-9 and abs(c + w / 2 - e1) < 1e-9


def test_z_edges_match_paper():
    g = _gold("paper_binning.json")
    for nb in (10, 5, 2):
        got = synth.equipopulated_edges(nb)
        assert np.max(np.abs(got - np.array(g["z_edges_%d" % nb]))) < 0.006


def test_ell_cut_keeps_bins_below():
    _, cen, _ = oracle.ell_bins(10.0, 5000.0, 15)
    assert [oracle.n_ell_used(cen, c) for c in (1000, 3000, 5000)] == [11, 14, 15]


# ------------------------------------------------------------------ interpolation
def test_interp_exact_on_power_law():
    k = np.exp(np.linspace(-5, 3, 97))
    for alpha in (-2.3, 0.0, 1.7):
        row = 3.5 * k ** alpha
        for kk in (k[0], 0.0123, 0.77, 5.5, k[-1]):
            assert oracle.interp(k, row, kk) == pytest.approx(3.5 * kk ** alpha, rel=1e-13)
            assert oracle.neff(k, row, kk) == pytest.approx(alpha, rel=1e-12, abs=1e-12)


def test_interp_at_nodes_and_out_of_range():
    k = np.exp(np.linspace(-3, 2, 11))
    row = np.exp(np.sin(np.arange(11.0)))
    for j in range(11):
        assert oracle.interp(k, row, k[j]) == pytest.approx(row[j], rel=1e-14)
    assert math.isnan(oracle.interp(k, row, k[0] * 0.999))
    assert math.isnan(oracle.interp(k, row, k[-1] * 1.001))
    oracle.lib().or_clear_error()


# ------------------------------------------------------------------ F2 and tree level
def test_F2_special_values():
    assert oracle.F2(1.0, 1.0, 1.0) == pytest.approx(2.0 / 7.0, rel=1e-15)        # equilateral
    assert oracle.F2(1.0, 1.0, 1e-9) == pytest.approx(0.0, abs=1e-12)               # mu = -1
    assert oracle.F2(1.0, 1.0, 2.0) == pytest.approx(2.0, rel=1e-15)                # mu = +1
    assert oracle.F2(0.7, 1.3, 1.1) == pytest.approx(oracle.F2(1.3, 0.7, 1.1), rel=1e-15)
    # right angle: mu = 0 -> 5/7
    assert oracle.F2(3.0, 4.0, 5.0) == pytest.approx(5.0 / 7.0, rel=1e-15)


# ------------------------------------------------------------------ halo integrals
def _tiny_tables(n_m=3, n_k=9):
    """Three masses, u known exactly at the table nodes."""
    t = synth.power_law_tables(n_z=2, n_chi=4, n_m=n_m, n_k=n_k)
    t.m = np.array([1e12, 3e12, 2e13])[:n_m]
    t.w_m = np.array([0.25, 0.5, 0.25])[:n_m] * t.m
    t.n_m = np.array([2e-13, 7e-14, 1e-15])[:n_m]
    t.u = np.exp(-0.5 * (t.k[None, :] * np.array([0.3, 0.6, 1.2])[:n_m, None]) ** 2)
    t.b1 = np.array([0.8, 1.1, 2.5])[:n_m]
    t.b2 = np.array([-0.3, 0.1, 1.9])[:n_m]
    return t


def test_halo_integral_brute_force():
    t = _tiny_tables()
    o = oracle.Oracle(t)
    rho = Fraction(t.cfg["rho_mean"])
    for mu, beta, idx in ((1, 1, [2]), (2, 0, [1, 4]), (3, 1, [0, 3, 8]), (2, 2, [5, 5])):
        ks = t.k[idx]
        exact = Fraction(0)
        for m in range(3):
            b = {0: Fraction(1), 1: Fraction(t.b1[m]), 2: Fraction(t.b2[m])}[beta]
            x = Fraction(t.w_m[m]) * b * (Fraction(t.m[m]) / rho) ** mu * Fraction(t.n_m[m])
            for j in idx:
                x *= Fraction(t.u[m, j])
            exact += x
        assert o.halo_I(mu, beta, ks) == pytest.approx(float(exact), rel=1e-13)


# ------------------------------------------------------------------ 3-D spectra structure
def _uniform_profile_oracle(alpha=-1.5, amp=1e4):
    t = synth.power_law_tables(alpha=alpha, amp=amp, n_chi=8)
    return oracle.Oracle(t), t


def test_power_spectrum_structure_and_response():
    o, t = _uniform_profile_oracle()
    # u = 1 and b1 = 1: I_1^1 = 1 by the mass normalisation, I_2^1 = I_2^0
    I11 = o.halo_I(1, 1, [0.1])
    assert I11 == pytest.approx(1.0, rel=1e-13)
    I20 = o.halo_I(2, 0, [0.1, 0.1])
    for k in (0.05, 0.3, 2.0):
        P = 1e4 * k ** -1.5
        X, R = o.spectrum(0, [k])
        assert X == pytest.approx(I20 + P, rel=1e-12)          # 1-halo + 2-halo
        assert R == pytest.approx((47.0 / 21.0 + 1.5 / 3.0) * P + I20, rel=1e-12)


def test_bispectrum_equilateral_polynomial():
    """With u = 1 the equilateral B_HM and R_B are polynomials in P(k): the P^2
    coefficients are 3 * 2 * F2_eq = 12/7 and the closed-form response."""
    alpha = -1.5
    o, t = _uniform_profile_oracle(alpha=alpha)
    I20 = o.halo_I(2, 0, [0.1, 0.1])
    I30 = o.halo_I(3, 0, [0.1, 0.1, 0.1])
    ks = np.array([0.04, 0.1, 0.3, 0.9, 2.5])
    P = 1e4 * ks ** alpha
    XB = np.array([o.spectrum(0, [k, k, k])[0] for k in ks])
    RB = np.array([o.spectrum(0, [k, k, k])[1] for k in ks])
    cX = np.polyfit(P, XB, 2)
    assert cX[0] == pytest.approx(12.0 / 7.0, rel=1e-8)
    assert cX[1] == pytest.approx(3.0 * I20, rel=1e-7)
    assert XB[0] - 12.0 / 7.0 * P[0] ** 2 - 3.0 * I20 * P[0] == pytest.approx(I30, rel=1e-8)
    # response: 433/126 B_PT + 5/126 B_G2 - (1/3) dilation, B_G2 = 2 * 3 * (1/4 - 1) P^2,
    # dilation = 3 pairs * 2 F2 * P^2 * 2 alpha
    quad = 433.0 / 126.0 * 12.0 / 7.0 + 5.0 / 126.0 * (-4.5) - (3 * 2 * 2.0 / 7.0 * 2 * alpha) / 3.0
    lin = 3.0 * I20 * (47.0 / 21.0 - alpha / 3.0)
    assert np.allclose(RB, quad * P ** 2 + lin * P + I30, rtol=1e-11)


def test_bispectrum_right_isosceles_closed_form():
    """Right isosceles triangle k1 = k2 = k, k3 = sqrt(2) k (k1 perpendicular to
    k2): from the geometry alone the cosines are mu_12 = 0 and mu_13 = mu_23 =
    -1/sqrt(2), so F2(k1, k2) = 5/7 and F2(k1, k3) = F2(k2, k3) = 5/7 - 3/4 + 1/7
    = 3/28, and the tidal kernel mu^2 - 1 is -1 on the perpendicular pair and
    -1/2 on the other two.  With u = 1 and b1 = 1 (I_1^1 = 1, I_2^1 = I_2^0,
    I_3^1 = I_3^0, b2 = 0 so I_2^2 = 0) and P = A k^alpha, the tree-level
    bispectrum and its response (eq. RespB under the tidal-kernel reading of
    B_G2, with the dilation sum_i dB_PT/dln k_i = 2 alpha B_PT of a power law)
    follow in closed form.  Unlike the equilateral case, every pair of legs has
    its own cosine here, so a cosine taken between the wrong legs fails."""
    alpha = -1.3
    o, _ = _uniform_profile_oracle(alpha=alpha)
    I20 = o.halo_I(2, 0, [0.1, 0.1])
    I30 = o.halo_I(3, 0, [0.1, 0.1, 0.1])
    r2 = math.sqrt(2.0)
    for k in (0.05, 0.2, 0.7):
        kv = [k, k, r2 * k]
        P1 = 1e4 * k ** alpha
        P3 = 1e4 * (r2 * k) ** alpha
        b_pt = 2.0 * (5.0 / 7.0 * P1 * P1 + 2.0 * 3.0 / 28.0 * P1 * P3)
        b_g2 = 2.0 * (-1.0 * P1 * P1 + 2.0 * (-0.5) * P1 * P3)
        X, R = o.spectrum(0, kv)
        assert X == pytest.approx(b_pt + I20 * (2.0 * P1 + P3) + I30, rel=1e-11)
        r_lin = (47.0 / 21.0 - alpha / 3.0) * (2.0 * P1 + P3)
        want = 433.0 / 126.0 * b_pt + 5.0 / 126.0 * b_g2 - 2.0 * alpha * b_pt / 3.0 + I20 * r_lin + I30
        assert R == pytest.approx(want, rel=1e-11)


def test_bispectrum_scaling_generic_triangle():
    """For P = A k^alpha the tree-level part scales as lambda^(2 alpha)."""
    alpha = -1.2
    o, _ = _uniform_profile_oracle(alpha=alpha)
    I20 = o.halo_I(2, 0, [0.1, 0.1]); I30 = o.halo_I(3, 0, [0.1, 0.1, 0.1])
    k = np.array([0.2, 0.3, 0.45])
    def tree(lam):
        kk = lam * k
        P = 1e4 * kk ** alpha
        return o.spectrum(0, list(kk))[0] - I30 - I20 * P.sum()
    ratio = tree(2.0) / tree(1.0)
    assert ratio == pytest.approx(2.0 ** (2 * alpha), rel=1e-11)
    # and equals sum over pairs of 2 F2 P_i P_j
    P = 1e4 * k ** alpha
    want = sum(2 * oracle.F2(k[i], k[j], k[3 - i - j]) * P[i] * P[j] for i, j in ((0, 1), (1, 2), (0, 2)))
    assert tree(1.0) == pytest.approx(want, rel=1e-11)


def test_kmax_cut_zeroes_integrand():
    t = synth.make_tables("tiny")
    o = oracle.Oracle(t)
    X, R = o.spectrum(3, [51.0 * 0 + t.cfg["k_max"] * 1.0001])
    assert X == 0.0 and R == 0.0


# ------------------------------------------------------------------ projection
def _light_halo_tables(alpha, n_chi, chi_max=3000.0, w=1e-3, amp=1e4):
    """Power-law P, constant kernels, u = 1 and very light haloes: I_1^1 = 1
    exactly (mass normalisation, b1 = 1) while every mass integral of higher
    order is O(m/rho) ~ 1e-10, so only the 2- and 3-halo (linear and tree)
    parts survive."""
    t = synth.power_law_tables(alpha=alpha, amp=amp, w_const=w, n_chi=n_chi, chi_max=chi_max)
    t.m = np.array([5.0, 9.0])
    t.w_m = np.array([0.5, 0.5]) * t.m
    rho = t.cfg["rho_mean"]
    t.n_m = np.ones(2) / np.sum(t.w_m * t.m / rho)
    t.u = np.ones((2, len(t.k)))
    return t


def test_projection_closed_form_power_spectrum():
    """eq. nProjection with P = A k^-3: P_ij(l) = W^2 A l^-3 sum_n w chi_n
    (chi^(2-2n) = chi^-2 times (l/chi)^-3), and the midpoint rule integrates the
    linear integrand exactly: sum = chi_max^2 / 2.  The response is
    (47/21 + 1) times the same (n_eff = -3)."""
    alpha, amp, w, X = -3.0, 1e4, 1e-3, 3000.0
    t = _light_halo_tables(alpha, 40, X, w, amp)
    o = oracle.Oracle(t)
    d, r = o.data_vector()
    for a in np.where(o.rows["kind"] == 2)[0]:
        l = o.centres[o.rows["lbin"][a][0]]
        want = w * w * amp * l ** alpha * X ** 2 / 2.0
        assert d[a] == pytest.approx(want, rel=1e-8)
        assert r[a] == pytest.approx((47.0 / 21.0 + 1.0) * want, rel=1e-8)


def test_projection_closed_form_bispectrum():
    """Bispectrum rows: B = sum_pairs 2 F2 P_i P_j ~ chi^6, projected with chi^-4
    gives sum_n w chi^2 = X^3/3 - X dchi^2/12 exactly (midpoint rule on a
    quadratic).  Equilateral response: 433/126 * 12/7 - 5/126 * 9/2 - (2 alpha/3) 12/7."""
    alpha, amp, w, X, n_chi = -3.0, 1e4, 1e-3, 3000.0, 40
    t = _light_halo_tables(alpha, n_chi, X, w, amp)
    o = oracle.Oracle(t)
    d, r = o.data_vector()
    dchi = X / n_chi
    s2 = X ** 3 / 3.0 - X * dchi ** 2 / 12.0
    seen_eq = False
    for a in np.where(o.rows["kind"] == 3)[0]:
        ls = [o.centres[b] for b in o.rows["lbin"][a]]
        tree = sum(2 * oracle.F2(ls[i], ls[j], ls[3 - i - j]) * ls[i] ** alpha * ls[j] ** alpha
                   for i, j in ((0, 1), (1, 2), (0, 2)))
        want = w ** 3 * amp ** 2 * tree * s2
        assert d[a] == pytest.approx(want, rel=1e-8)
        if ls[0] == ls[1] == ls[2]:
            seen_eq = True
            c = 433.0 / 126.0 * 12.0 / 7.0 - 5.0 / 126.0 * 4.5 - 2.0 * alpha / 3.0 * 12.0 / 7.0
            assert r[a] == pytest.approx(c * w ** 3 * amp ** 2 * 12.0 / 7.0 * ls[0] ** (2 * alpha) * s2 / (12.0 / 7.0), rel=1e-8)
    assert seen_eq


# ------------------------------------------------------------------ one-halo
def test_one_halo_is_gram_of_factor():
    """(1/Omega) A A^T with A[a,(n,m)] = sqrt(w_n w_m n_m) chi^-(2p-1) prod W
    (m/rho)^p prod u equals the oracle's literal entry (eq. General1h)."""
    t = synth.make_tables("tiny", n_chi=16, n_m=8)
    o = oracle.Oracle(t)
    rows = o.rows
    ell, U = o.u_table()
    N = o.N
    A = np.zeros((N, o.n_chi * o.n_m))
    for a in range(N):
        p = int(rows["kind"][a])
        legs = [rows["lbin"][a][0]] * 2 if p == 2 else list(rows["lbin"][a])
        for n in range(o.n_chi):
            chi = t.chi[n]
            if max(ell[b] for b in legs) / chi > t.cfg["k_max"]:
                continue
            tw = math.sqrt(t.w_chi[n]) * chi ** -(2 * p - 1)
            for z in rows["zbin"][a][:p]:
                tw *= t.W[z, n]
            for m in range(o.n_m):
                v = tw * math.sqrt(t.w_m[m] * t.n_m[m]) * (t.m[m] / t.cfg["rho_mean"]) ** p
                for b in legs:
                    v *= U[b, n, m]
                A[a, n * o.n_m + m] = v
    G = A @ A.T / o.omega
    rng = np.random.default_rng(3)
    pairs = np.stack([rng.integers(0, N, 300), rng.integers(0, N, 300)], 1)
    got = o.cov1h_pairs(pairs)
    want = G[pairs[:, 0], pairs[:, 1]]
    assert np.max(np.abs(got - want) / np.abs(want)) < 1e-12


def test_one_halo_closed_form_single_mass():
    """One mass, u = 1, constant kernels: C_1h = (1/Omega) w n (m/rho)^n W^n
    sum_chi w chi^(2-2n), n = p_a + p_b legs (4, 5 or 6)."""
    t = synth.power_law_tables(n_z=2, n_chi=16, n_m=1, w_const=2e-3)
    o = oracle.Oracle(t)
    rows = o.rows
    iP = int(np.where(rows["kind"] == 2)[0][0]); iB = int(np.where(rows["kind"] == 3)[0][0])
    for a, b, n in ((iP, iP, 4), (iB, iP, 5), (iB, iB, 6)):
        want = (t.w_m[0] * t.n_m[0] * (t.m[0] / t.cfg["rho_mean"]) ** n * 2e-3 ** n
                * np.sum(t.w_chi * t.chi ** (2.0 - 2.0 * n)) / o.omega)
        assert o.cov1h_pairs(np.array([[a, b]]))[0] == pytest.approx(want, rel=1e-12)


# ------------------------------------------------------------------ Gaussian
def test_gaussian_single_bin_textbook():
    """One redshift bin: Var(P) = 2 P_s^2 / N(l); Var(B) = (Omega/N_tri) s P1 P2 P3
    with s = 6, 2, 1 for equilateral, isosceles, scalene triangles."""
    t = synth.make_tables("tiny", n_z=1)
    o = oracle.Oracle(t)
    ps = o.ps_table()
    nm = o.nmodes(); nt = o.ntri()
    rows = o.rows
    N = o.N
    diag = o.gauss_pairs(np.stack([np.arange(N), np.arange(N)], 1))
    for a in range(N):
        if rows["kind"][a] == 2:
            b = rows["lbin"][a][0]
            assert diag[a] == pytest.approx(2 * ps[b, 0, 0] ** 2 / nm[b], rel=1e-14)
        else:
            i, j, k = rows["lbin"][a]
            s = 6 if i == j == k else (2 if (i == j or j == k) else 1)
            want = o.omega / nt[rows["tri"][a]] * s * ps[i, 0, 0] * ps[j, 0, 0] * ps[k, 0, 0]
            assert diag[a] == pytest.approx(want, rel=1e-14)
    # different ell-bins / triangles and P-B pairs are uncorrelated
    pb = np.array([[N - 1, 0], [1, 0], [N - 1, N - 2]])
    assert np.all(o.gauss_pairs(pb) == 0.0)


def test_gaussian_tomographic_power_spectrum():
    """Knox tomographic form: Cov[P_ij, P_ij] = (P_ii P_jj + P_ij^2)/N and
    Cov[P_ii, P_jj] = 2 P_ij^2 / N."""
    t = synth.make_tables("tiny", n_z=3)
    o = oracle.Oracle(t)
    ps = o.ps_table(); nm = o.nmodes()
    rows = o.rows
    idx = {(int(rows["lbin"][a][0]), int(rows["zbin"][a][0]), int(rows["zbin"][a][1])): a
           for a in range(o.N) if rows["kind"][a] == 2}
    b = 2
    a01, a00, a11 = idx[(b, 0, 1)], idx[(b, 0, 0)], idx[(b, 1, 1)]
    g = o.gauss_pairs(np.array([[a01, a01], [a11, a00]]))
    assert g[0] == pytest.approx((ps[b, 0, 0] * ps[b, 1, 1] + ps[b, 0, 1] ** 2) / nm[b], rel=1e-14)
    assert g[1] == pytest.approx(2 * ps[b, 0, 1] ** 2 / nm[b], rel=1e-14)


def test_shot_noise_value():
    t = synth.make_tables("tiny")
    o = oracle.Oracle(t)
    nbar = 30.0 * (60 * 180 / math.pi) ** 2 / 2
    assert o.shot_noise() == pytest.approx(0.09 / nbar, rel=1e-14)


# ------------------------------------------------------------------ whole covariance
@pytest.fixture(scope="module")
def tiny_run():
    t = synth.make_tables("tiny")
    o = oracle.Oracle(t)
    return o, o.run()


def test_covariance_symmetric_psd(tiny_run):
    o, res = tiny_run
    C = res["C"]
    assert np.array_equal(C, C.T)
    s = np.sqrt(np.diag(C))
    ev = np.linalg.eigvalsh(C / np.outer(s, s))
    assert ev.min() > 0
    # each term on its own is PSD; the super-sample term is rank one
    _, r = o.data_vector()
    ssc = o.cfg["sigma_b2"] * np.outer(r, r)
    ev2 = np.linalg.eigvalsh(ssc / np.outer(s, s))
    assert ev2[-2] < 1e-12 * ev2[-1]


def test_pairs_match_full(tiny_run):
    o, res = tiny_run
    pairs = synth.sample_pairs(o.N, 500, seed=7)
    got = o.cov_pairs(pairs)
    want = res["C"][pairs[:, 0], pairs[:, 1]]
    assert np.max(np.abs(got - want) / np.abs(want)) < 1e-13


def test_bin_permutation_invariance_bitwise(tiny_run):
    """Rows that differ only by a permutation of redshift bins (same
    ell-configuration) carry bitwise-identical data-vector values and
    one-halo covariances (Limber: every bin sees the same chi)."""
    o, res = tiny_run
    rows = o.rows
    d = res["d"]
    canon, reps = oracle.canonical_rows(rows)
    groups = {}
    for a, c in enumerate(canon):
        groups.setdefault(int(c), []).append(a)
    multi = [g for g in groups.values() if len(g) > 1]
    assert multi
    for g in multi:
        assert len({d[a] for a in g}) == 1
    g = multi[0]
    other = [0, 5, o.N - 1]
    vals = [o.cov1h_pairs(np.array([[a, b] for b in other])) for a in g]
    for v in vals[1:]:
        assert np.array_equal(v, vals[0])


def test_snr_matches_library_solve(tiny_run):
    o, res = tiny_run
    C, d = res["C"], res["d"]
    want = float(d @ np.linalg.solve(C, d))
    assert res["snr2"] == pytest.approx(want, rel=1e-10)


def test_snr_power_of_two_scaling_bitwise(tiny_run):
    o, res = tiny_run
    C, d = res["C"], res["d"]
    s = np.random.default_rng(1).integers(-40, 40, size=len(d))
    sc = np.ldexp(1.0, s)
    C2 = C * sc[:, None] * sc[None, :]
    d2 = d * sc
    assert oracle.Oracle.snr2(C2, d2) == res["snr2"]


def test_snr_sorted_not_above_paper():
    t = synth.make_tables("tiny")
    paper = oracle.Oracle(t).run()["snr2"]
    srt = oracle.Oracle(t, tomo="sorted").run()["snr2"]
    assert srt <= paper * (1 + 1e-12)


def test_snr_diagonal_case():
    rng = np.random.default_rng(0)
    c = rng.uniform(0.5, 2.0, 50); d = rng.normal(size=50)
    assert oracle.Oracle.snr2(np.diag(c), d) == pytest.approx(np.sum(d * d / c), rel=1e-14)
    with pytest.raises(np.linalg.LinAlgError):
        oracle.Oracle.snr2(-np.eye(3), np.ones(3))


# ------------------------------------------------------------------ counts
def test_closed_form_counts():
    nm = oracle.n_modes([500.0], [100.0], 0.36)
    assert nm[0] == pytest.approx(2 * 500 * 100 * 0.36)
    with pytest.raises(ValueError):
        oracle.n_tri_closed(1.0, 1.0, 2.0, 0.1, 0.1, 0.1, 0.36)


def test_lattice_mode_counts_match_continuum():
    """Lattice mode counts follow N(l) = 2 l Delta l f_sky (Sec. 3.2.2)."""
    edges, cen, wid = oracle.ell_bins(100.0, 1000.0, 5)
    thr = oracle.lattice_thresholds(edges, 0.36)
    for b in range(5):
        got = oracle.lattice_modes(thr, b)
        assert got == pytest.approx(2 * cen[b] * wid[b] * 0.36, rel=2e-3)
    # bins partition the annulus: the sum equals a direct count of all points
    tot = sum(oracle.lattice_modes(thr, b) for b in range(5))
    R = int(math.isqrt(thr[-1])) + 1
    direct = sum(1 for x in range(-R, R + 1) for y in range(-R, R + 1) if thr[0] <= x * x + y * y < thr[-1])
    assert tot == direct


def test_lattice_triangles_brute_force_small():
    """Pair counting against an independent loop over all three vectors on a
    coarse lattice."""
    thr = [4, 16, 40, 90]
    def modes(lo, hi):
        R = int(math.isqrt(hi)) + 1
        return [(x, y) for x in range(-R, R + 1) for y in range(-R, R + 1) if lo <= x * x + y * y < hi]
    for b1, b2, b3 in ((0, 0, 0), (0, 1, 1), (1, 1, 2), (0, 2, 2), (1, 2, 2)):
        q1s = modes(thr[b1], thr[b1 + 1]); q2s = modes(thr[b2], thr[b2 + 1]); q3s = set(modes(thr[b3], thr[b3 + 1]))
        want = sum(1 for a in q1s for b in q2s if (-(a[0] + b[0]), -(a[1] + b[1])) in q3s)
        assert oracle.lattice_triangles(thr, b1, b2, b3) == want


def test_lattice_triangles_near_closed_form():
    """For well-formed (non-flat) triangles the lattice count is close to the
    bin-centre continuum count (App. B)."""
    edges, cen, wid = oracle.ell_bins(100.0, 1000.0, 5)
    thr = oracle.lattice_thresholds(edges, 0.36)
    for (i, j, k) in ((0, 0, 0), (1, 1, 1), (0, 1, 1)):
        lat = oracle.lattice_triangles(thr, i, j, k)
        cf = oracle.n_tri_closed(cen[i], cen[j], cen[k], wid[i], wid[j], wid[k], 0.36)
        assert 0.85 < lat / cf < 1.15


def test_bispectrum_symmetric_under_leg_permutation():
    """The bispectrum and its response are symmetric functions of the three
    legs; a wrong index in any cyclic term breaks this."""
    from itertools import permutations
    t = synth.make_tables("tiny")
    t.b1 = np.linspace(0.7, 3.0, len(t.m))
    t.b2 = np.linspace(-0.4, 2.0, len(t.m))
    o = oracle.Oracle(t)
    for n, kv in ((10, [0.11, 0.17, 0.23]), (40, [0.05, 0.09, 0.12]), (60, [0.02, 0.03, 0.045])):
        vals = [o.spectrum(n, list(p)) for p in permutations(kv)]
        X0, R0 = vals[0]
        assert X0 > 0
        for X, R in vals[1:]:
            assert X == pytest.approx(X0, rel=1e-13)
            assert R == pytest.approx(R0, rel=1e-13)


@pytest.mark.parametrize("preset", ["tiny", "mid"])
def test_snr_lmax_curve_matches_cut_vectors(preset):
    """(S/N)^2(ell_max) from one Cholesky in ell_max order equals, at every
    cut, the S/N of a separately planned data vector cut at that ell_max
    (its own enumeration, covariance and Cholesky)."""
    t = synth.make_tables(preset)
    o = oracle.Oracle(t)
    ref = o.run()
    curve = o.snr2_lmax(ref["C"], ref["d"])
    assert abs(curve[-1] - ref["snr2"]) <= 1e-12 * ref["snr2"]
    assert np.all(np.diff(curve) > 0)
    c = o.centres
    for b in range(o.n_ell - 1):
        tb = synth.make_tables(preset, ell_cut=0.5 * (c[b] + c[b + 1]))
        ob = oracle.Oracle(tb)
        assert ob.n_ell == b + 1
        assert abs(curve[b] - ob.run()["snr2"]) <= 1e-10 * curve[b]
