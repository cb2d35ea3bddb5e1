"""Pins of the oracle's bin averaging: sub-bin weights of power-spectrum and
triangle bins (the mode and triangle counts of Sec. 3.2.2 and App. B), and
the averaged data vector and one-halo covariance."""
import ctypes as ct
import math

import numpy as np
import pytest

import oracle
import synth


def _lib():
    L = oracle.lib()
    L.or_lattice_mode_moment.restype = ct.c_double
    L.or_lattice_mode_moment.argtypes = [ct.c_int64, ct.c_int64, ct.c_int]
    L.or_lattice_triangle_moment.restype = ct.c_double
    L.or_lattice_triangle_moment.argtypes = [ct.c_int64] * 6 + [ct.c_int, ct.POINTER(ct.c_double)]
    return L


def test_power_weights_match_lattice_modes():
    """The sub-bin weights of a power-spectrum bin (proportional to l) give
    the mean of l^4 over the bin's lattice modes to 3e-3; uniform weights
    miss it by about 6 %."""
    f_sky, S = 0.36, 16
    edges, centres, _ = oracle.ell_bins(100.0, 1000.0, 5)
    thr = oracle.lattice_thresholds(edges, f_sky)
    lf = 2.0 * math.pi / math.sqrt(4.0 * math.pi * f_sky)
    sub = oracle.sub_bin_centres(edges, centres, 5, S)
    lists = oracle.averaging_lists([2] * 5, [(b, b, -1) for b in range(5)], S, sub, None)
    for b, (L, W) in enumerate(lists):
        n = oracle.lattice_modes(thr, b)
        lattice = _lib().or_lattice_mode_moment(thr[b], thr[b + 1], 2) / n * lf ** 4
        ls = np.array(sub)[L[:, 0]]
        assert abs(np.sum(W * ls ** 4) / lattice - 1.0) < 3e-3
        assert abs(np.mean(ls ** 4) / lattice - 1.0) > 0.04
        assert abs(np.sum(W) - 1.0) < 1e-15


def test_cell_count_small_cell_limit():
    """For a small cell far from flat triangles the continuum pair count is
    the closed-form density 4 l1 l2 l3 / Lambda times the cell volume (the
    count N_tri of App. B without its constant (Omega / (2 pi)^2)^2 2 pi)."""
    l1, l2, l3, h = 300.0, 400.0, 500.0, 0.5
    got = oracle.cell_pairs(l1 - h, l1 + h, l2 - h, l2 + h, l3 - h, l3 + h)
    om = 4.0 * math.pi * 0.36
    closed = oracle.n_tri_closed(l1, l2, l3, 2 * h, 2 * h, 2 * h, 0.36) / ((om / (2 * math.pi) ** 2) ** 2 * 2 * math.pi)
    assert abs(got / closed - 1.0) < 1e-4


@pytest.fixture(scope="module")
def fine_lattice():
    """Ordered mode pairs of the scalene bin of three ell-bins over 30-120,
    on a lattice of fundamental 0.5 (fine enough to stand in for the
    continuum): pair count and mean of (l1 l2 l3)^2."""
    edges, centres, widths = oracle.ell_bins(30.0, 120.0, 3)
    lf = 0.5
    thr = [int(math.ceil((e / lf) ** 2)) for e in edges]
    t = (0, 1, 2)
    mom = ct.c_double()
    cnt = _lib().or_lattice_triangle_moment(thr[0], thr[1], thr[1], thr[2], thr[2], thr[3], 1, ct.byref(mom))
    return dict(edges=edges, centres=centres, widths=widths, lf=lf, t=t, count=cnt,
                mean=mom.value / cnt * lf ** 6)


def test_cell_count_matches_fine_lattice(fine_lattice):
    """Whole-bin continuum count vs the fine lattice (each lattice mode
    covers l_f^2 of the plane): within 1 %."""
    fl = fine_lattice
    e = fl["edges"]
    cont = oracle.cell_pairs(e[0], e[1], e[1], e[2], e[2], e[3], n=16) * 2.0 * math.pi / fl["lf"] ** 4
    assert abs(cont / fl["count"] - 1.0) < 1e-2


def test_triangle_weights_match_fine_lattice(fine_lattice):
    """The mean of (l1 l2 l3)^2 over the bin's triangles: cell-count weights
    at 16 sub-bins per side land within 2 % of the lattice, uniform weights
    about 8 % off."""
    fl = fine_lattice
    S = 16
    sub = oracle.sub_bin_centres(fl["edges"], fl["centres"], 3, S)
    (L, W), = oracle.averaging_lists([3], [fl["t"]], S, sub, fl["widths"])
    ls = np.array(sub)[L]
    f = (ls[:, 0] * ls[:, 1] * ls[:, 2]) ** 2
    assert abs(np.sum(W * f) / fl["mean"] - 1.0) < 2e-2
    assert abs(np.mean(f) / fl["mean"] - 1.0) > 5e-2


def test_equal_legs_symmetric_weights():
    """Swapping the sub-bins of two legs in one ell-bin leaves the weight
    unchanged (the cell count is symmetric in the two modes)."""
    edges, centres, widths = oracle.ell_bins(100.0, 1000.0, 5)
    S = 4
    sub = oracle.sub_bin_centres(edges, centres, 5, S)
    tris = [t[:3] for t in oracle.triangles(centres) if t[3] == "I" and t[0] == t[1]]
    for tri, (L, W) in zip(tris, oracle.averaging_lists([3] * len(tris), tris, S, sub, widths)):
        wt = {tuple(g): w for g, w in zip(L.tolist(), W)}
        for (a, b, c), w in wt.items():
            assert abs(wt[(b, a, c)] / w - 1.0) < 1e-12


@pytest.fixture(scope="module")
def tiny_tables():
    return synth.make_tables("tiny")


def test_averaging_path_at_centres(tiny_tables):
    """With one sub-bin the averaging code (entry lists, weighted sums, the
    double average of the one-halo term) reproduces the bin-centre code."""
    o = oracle.Oracle(tiny_tables)
    X, R = o.spectra()
    Xa, Ra = o.spectra_avg()
    assert np.array_equal(X, Xa) and np.array_equal(R, Ra)
    pairs = synth.sample_pairs(o.N, 300, seed=4)
    assert np.allclose(o.cov1h_avg_pairs(pairs), o.cov1h_pairs(pairs), rtol=1e-14, atol=0)


def test_converges_with_sub_bins(tiny_tables):
    """Power-spectrum rows converge at second order in 1 / n_sub (midpoint
    rule over smooth sub-bins)."""
    d = {S: oracle.Oracle(tiny_tables, n_sub=S).data_vector()[0] for S in (2, 4, 8)}
    o = oracle.Oracle(tiny_tables)
    P = o.rows["kind"] == 2
    e1 = np.max(np.abs(d[2][P] - d[4][P]) / np.abs(d[8][P]))
    e2 = np.max(np.abs(d[4][P] - d[8][P]) / np.abs(d[8][P]))
    assert e2 < e1 / 3.0
    # and the averages move away from the centre values
    assert np.max(np.abs(d[8] - o.data_vector()[0]) / np.abs(d[8])) > 1e-3


def test_averaged_one_halo_is_a_gram(tiny_tables):
    """The double average of the one-halo term is a Gram matrix of averaged
    factors: symmetric positive semi-definite on the distinct rows."""
    o = oracle.Oracle(tiny_tables, n_sub=2)
    canon, reps = oracle.canonical_rows(o.rows)
    ii, jj = np.meshgrid(reps, reps, indexing="ij")
    M = o.cov1h_pairs(np.stack([ii.ravel(), jj.ravel()], 1)).reshape(len(reps), len(reps))
    assert np.allclose(M, M.T, rtol=1e-13, atol=0)
    ev = np.linalg.eigvalsh(M)
    assert ev[0] > -1e-12 * ev[-1]
    with pytest.raises(ValueError):
        o.ngins_pairs(np.array([[0, 0]]))
