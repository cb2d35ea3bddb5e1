"""Pins of the bias-dependent pieces of the oracle's spectra and responses.

With a single halo mass and u = 1, every halo integral of eq. ImunuHalos
collapses to I_mu^beta = w n (m/rho)^mu b_beta, and the mass normalisation
w n (m/rho) = 1 gives I_1^1 = b1.  The response of eqs. PowerHMResp and
BispHMResp is then a polynomial in b1 and b2 whose coefficients follow from
the physics of each term, not from the oracle's code:

* the one-halo terms respond as the bias-weighted one-halo terms (reading
  of eq. ImunuHalosDeltaB: the long-mode derivative raises the bias order,
  I_mu^0 -> I_mu^1), so with a negligible linear power R_P = b1 P_1h and
  R_B = b1 B_1h;
* b2 enters only through the derivative of the two-halo bispectrum's
  I_2^1(k2, k3) (-> I_2^2), multiplied by I_1^1(k1) P(k1) of the lone leg;
* in b1 (b2 = 0) the equilateral response is a cubic whose b1 coefficient is
  the one-halo response, whose b1^2 coefficient is the two-halo part with the
  linear response R_lin = (47/21 - alpha/3) P of a power law, and whose b1^3
  coefficient is the tree-level response, where the dilation term of a
  power law is 2 alpha B_PT by homogeneity (B_PT(lambda k) = lambda^(2 alpha)
  B_PT(k)).
A mistake that swaps I_2^2 with I_2^1, or I_3^1 with I_3^0, or drops a bias
factor, fails one of these.  CPU only.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth


def _single_mass(b1, b2, alpha=-1.5, amp=1e4):
    t = synth.power_law_tables(n_z=2, n_chi=8, n_m=1, alpha=alpha, amp=amp)
    return dataclasses.replace(t, b1=np.array([float(b1)]), b2=np.array([float(b2)]))


def _mrho(t):
    return t.m[0] / t.cfg["rho_mean"]


def test_single_mass_normalisation():
    t = _single_mass(1.0, 0.0)
    assert t.w_m[0] * t.n_m[0] * _mrho(t) == pytest.approx(1.0, rel=1e-14)
    o = oracle.Oracle(t)
    for b1 in (0.5, 2.0):
        ob = oracle.Oracle(_single_mass(b1, 0.0))
        assert ob.halo_I(1, 1, [0.3]) == pytest.approx(b1, rel=1e-14)
        assert ob.halo_I(2, 1, [0.3, 0.3]) == pytest.approx(b1 * _mrho(t), rel=1e-14)
    assert o.halo_I(3, 0, [0.1, 0.2, 0.3]) == pytest.approx(_mrho(t) ** 2, rel=1e-14)


@pytest.mark.parametrize("b1,b2", [(0.6, -0.3), (1.7, 0.9), (3.2, 5.0)])
def test_one_halo_response_is_bias_weighted(b1, b2):
    """Negligible linear power: only the one-halo terms survive, and their
    long-mode response is b1 times the one-halo spectrum."""
    o = oracle.Oracle(_single_mass(b1, b2, amp=1e-30))
    for ks in ([0.2], [0.2, 0.2, 0.2], [0.15, 0.25, 0.33]):
        X, R = o.spectrum(0, ks)
        assert R / X == pytest.approx(b1, rel=1e-12)


def test_b2_enters_through_the_two_halo_response():
    """R_B(b2) - R_B(0) = b1 b2 (m/rho) sum_a P(k_a); b2 leaves P, B and R_P
    unchanged."""
    alpha, amp, b1 = -1.5, 1e4, 1.3
    ks = [0.15, 0.25, 0.33]
    P = amp * np.array(ks) ** alpha
    base = oracle.Oracle(_single_mass(b1, 0.0, alpha, amp))
    XB0, RB0 = base.spectrum(0, ks)
    XP0, RP0 = base.spectrum(0, [0.2])
    mr = _mrho(_single_mass(b1, 0.0))
    for b2 in (-0.7, 2.5):
        o = oracle.Oracle(_single_mass(b1, b2, alpha, amp))
        XB, RB = o.spectrum(0, ks)
        XP, RP = o.spectrum(0, [0.2])
        assert XB == XB0 and XP == XP0 and RP == RP0
        assert RB - RB0 == pytest.approx(b1 * b2 * mr * P.sum(), rel=1e-10)


def test_equilateral_response_cubic_in_b1():
    # an amplitude that keeps the three terms of one size, so that the
    # coefficients are well determined by three values of b1
    alpha, amp, k = -1.5, 1.0, 0.2
    P = amp * k ** alpha
    mr = _mrho(_single_mass(1.0, 0.0))
    b1s = np.array([0.5, 1.0, 2.0, 3.5])
    RB = np.array([oracle.Oracle(_single_mass(b, 0.0, alpha, amp)).spectrum(0, [k, k, k])[1] for b in b1s])
    # R = c1 b1 + c2 b1^2 + c3 b1^3: solve the 3 x 3 system from three values,
    # check the fourth
    V = np.stack([b1s, b1s ** 2, b1s ** 3], 1)
    c = np.linalg.solve(V[:3], RB[:3])
    assert V[3] @ c == pytest.approx(RB[3], rel=1e-12)
    B_pt = 12.0 / 7.0 * P ** 2                   # 3 pairs x 2 F2_eq, F2_eq = 2/7
    B_g2 = 2.0 * 3.0 * (0.25 - 1.0) * P ** 2    # mu = -1/2 (reading of B_G2)
    tree = 433.0 / 126.0 * B_pt + 5.0 / 126.0 * B_g2 - (2.0 * alpha * B_pt) / 3.0
    assert c[0] == pytest.approx(mr ** 2, rel=1e-10)                       # I_3^1 at b1 = 1
    assert c[1] == pytest.approx(3.0 * mr * (47.0 / 21.0 - alpha / 3.0) * P, rel=1e-10)
    assert c[2] == pytest.approx(tree, rel=1e-10)


def test_bias_recipe_consistency():
    """The synthetic b1 obeys sum_m w_m (M_m/rho) n_m b1_m = 1, so the
    large-scale limit of I_1^1 is 1 (eq. BoundinMass, beta = 1)."""
    t = synth.with_bias(synth.make_tables("tiny"))
    o = oracle.Oracle(t)
    assert o.halo_I(1, 1, [1e-4]) == pytest.approx(1.0, abs=1e-6)
    assert np.min(t.b2) < 0.0 < np.max(t.b2)
