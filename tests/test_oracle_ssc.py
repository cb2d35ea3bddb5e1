"""Pins of the oracle's super-sample term resolved along the line of sight:
sigma_W^2(chi) of the survey disk (eq. Mask in the thin-shell limit, App. B)
and the chi-resolved covariance of eq. WLSSCflatskyLimber."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import synth


def _flat_tables(P_of_k, n_chi=16, chi_max=3000.0, n_k=64):
    """Tables whose P(k, chi) = P_of_k(k) at every chi, on a k range wide
    enough that the disk window is resolved at every chi node."""
    t = synth.power_law_tables(n_chi=n_chi, chi_max=chi_max, n_k=n_k)
    theta = math.acos(1.0 - 2.0 * t.cfg["f_sky"])  # Omega = 2 pi (1 - cos Theta)
    k = np.exp(np.linspace(math.log(1e-5 / (chi_max * theta)), math.log(1e6 / (t.chi[0] * theta)), n_k))
    P = np.tile(P_of_k(k), (n_chi, 1))
    u = np.ones((len(t.m), n_k))
    return dataclasses.replace(t, k=k, P=P, u=u), theta


def test_white_noise_disk_variance():
    """Constant P = P0: the disk average of white noise has variance P0 over
    the disk's area pi (chi Theta)^2 (from int_0^inf J1(x)^2 / x dx = 1/2).  Truncation of the k range costs < 1e-6 here; the trapezoid
    rule aliases the unresolved oscillation of J1^2 at x >> 1 / h, which
    the tolerance bounds (a few 1e-5 at most)."""
    P0 = 2.5e3
    t, theta = _flat_tables(lambda k: np.full_like(k, P0))
    o = oracle.Oracle(t)
    assert abs(o.theta_sky() - theta) < 1e-15
    sw = o.sigma_w2()
    want = P0 / (math.pi * (t.chi * theta) ** 2)
    assert np.max(np.abs(sw / want - 1.0)) < 1e-4


def test_power_law_disk_variance():
    """P = A / k: sigma_W^2 = (2/pi) A / (chi Theta) int_0^inf J1(x)^2 / x^2 dx
    = 8 A / (3 pi^2 chi Theta) (Weber-Schafheitlin integral, lambda = 2)."""
    A = 40.0
    t, theta = _flat_tables(lambda k: A / k)
    sw = oracle.Oracle(t).sigma_w2()
    want = 8.0 * A / (3.0 * math.pi ** 2 * t.chi * theta)
    assert np.max(np.abs(sw / want - 1.0)) < 1e-4


def test_quadrature_converges():
    """Doubling the nodes changes the synthetic-table value by < 1e-6."""
    o = oracle.Oracle(synth.make_tables("tiny"))
    a = o.sigma_w2()
    b = o.sigma_w2(2 * oracle.Oracle.SIGMA_W_NODES)
    assert np.all(a > 0.0)
    assert np.max(np.abs(a / b - 1.0)) < 1e-6


def test_variance_falls_with_distance():
    """Synthetic tables: the disk grows with chi and the growth factor falls,
    so sigma_W^2 decreases monotonically along the line of sight."""
    sw = oracle.Oracle(synth.make_tables("tiny")).sigma_w2()
    assert np.all(np.diff(sw) < 0.0)


@pytest.fixture(scope="module")
def tiny():
    return oracle.Oracle(synth.make_tables("tiny"))


def test_sum_of_slab_rank_ones(tiny):
    """The chi-resolved term is a sum over slabs of independent long modes:
    with r^(n) the projected response restricted to node n (the pinned
    projection with every kernel zeroed off that node),
        C_ssc = sum_n sigma_W^2(chi_n) / w_n  r^(n) r^(n)T."""
    o = tiny
    sw = o.sigma_w2()
    N = o.N
    want = np.zeros((N, N))
    for n in range(o.n_chi):
        W = np.zeros_like(o.t.W)
        W[:, n] = o.t.W[:, n]
        _, rn = oracle.Oracle(dataclasses.replace(o.t, W=W)).data_vector()
        want += sw[n] / o.t.w_chi[n] * np.outer(rn, rn)
    ii, jj = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    got = o.ssc_chi_pairs(np.stack([ii.ravel(), jj.ravel()], 1), sw=sw).reshape(N, N)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-15 * np.max(np.abs(want)))


def test_psd_rank_and_full_matrix(tiny):
    """Positive semi-definite, rank <= N_chi, and the full-matrix route
    (covariance with ssc="chi") agrees with the pairwise one."""
    o = tiny
    N = o.N
    ii, jj = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    pairs = np.stack([ii.ravel(), jj.ravel()], 1)
    S = o.ssc_chi_pairs(pairs).reshape(N, N)
    ev = np.linalg.eigvalsh(S)
    assert ev[0] >= -1e-12 * ev[-1]
    assert np.sum(ev > 1e-12 * ev[-1]) <= o.n_chi
    C = o.covariance(ssc="chi")
    want = o.cov_pairs(pairs, ssc="chi").reshape(N, N)
    assert np.allclose(C, want, rtol=1e-12, atol=0)
    assert np.array_equal(C, C.T)
