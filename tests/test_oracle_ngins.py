"""Pins of the oracle's B.B, P.T and P.B in-survey terms (eqs. CovBB and
Covpb of App. B) and of its projected one-halo trispectrum."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def tiny():
    return oracle.Oracle(synth.make_tables("tiny"))


@pytest.fixture(scope="module")
def one_bin():
    return oracle.Oracle(synth.make_tables("tiny", n_z=1))


def test_trispectrum_matches_power_spectrum_one_halo(tiny):
    """At legs (l, l, l', l') the projected one-halo trispectrum is Omega times
    the one-halo power-spectrum covariance (eq. CovPPNG), which the oracle
    computes by a separate routine pinned by brute force."""
    o = tiny
    P = np.where(o.rows["kind"] == 2)[0]
    rng = np.random.default_rng(3)
    for _ in range(20):
        a, b = rng.choice(P, 2)
        la, lb = o.rows["lbin"][a][0], o.rows["lbin"][b][0]
        za, zb = o.rows["zbin"][a][:2], o.rows["zbin"][b][:2]
        t4 = o.trispec([la, la, lb, lb], [za[0], za[1], zb[0], zb[1]])
        c1h = o.cov1h_pairs(np.array([[a, b]]))[0]
        assert abs(t4 - o.omega * c1h) <= 1e-13 * abs(t4)


def test_symmetric(tiny):
    o = tiny
    pairs = synth.sample_pairs(o.N, 400, seed=5)
    v = o.ngins_pairs(pairs)
    w = o.ngins_pairs(pairs[:, ::-1].copy())
    assert np.allclose(v, w, rtol=1e-13, atol=0)  # the sums run in another order
    assert np.count_nonzero(v) > 50


def test_equal_legs_exchange(tiny):
    """For a triangle with two legs in one bin, exchanging the bins on those
    legs describes the same statistic: every term must be unchanged."""
    o = tiny
    tris = o.rows["triangles"]
    t = next(q for q, tr in enumerate(tris) if tr[0] == tr[1] != tr[2])
    l1, l2, l3 = tris[t][:3]
    rows = dict(kind=[], lbin=[], zbin=[], tri=[])
    for z in [(0, 1, 1), (1, 0, 1), (0, 1, 0), (1, 0, 0)]:
        rows["kind"].append(3); rows["lbin"].append((l1, l2, l3)); rows["zbin"].append(z); rows["tri"].append(t)
    n0 = len(rows["kind"])
    for a in range(o.N):  # every data-vector row as a partner
        for key in ("kind", "lbin", "zbin", "tri"):
            rows[key].append(o.rows[key][a])
    rows = {k: np.array(v, np.int32) for k, v in rows.items()}
    partners = np.arange(n0, n0 + o.N)
    for x, y in [(0, 1), (2, 3)]:
        vx = o.ngins_pairs(np.stack([np.full(o.N, x), partners], 1), rows)
        vy = o.ngins_pairs(np.stack([np.full(o.N, y), partners], 1), rows)
        assert np.allclose(vx, vy, rtol=1e-14, atol=0) and np.count_nonzero(vx) > 0


def test_one_bin_power_bispectrum_closed_form(one_bin):
    """n_z = 1: each bispectrum leg in the power spectrum's bin gives
    2 P^s(l) B / N(l) (the two printed terms coincide)."""
    o = one_bin
    d, _ = o.data_vector()
    ps, nm = o.ps_table(), o.nmodes()
    P = np.where(o.rows["kind"] == 2)[0]
    B = np.where(o.rows["kind"] == 3)[0]
    pairs = np.array([(a, b) for a in P for b in B])
    got = o.ngins_pairs(pairs)
    for (a, b), g in zip(pairs, got):
        l = o.rows["lbin"][a][0]
        m = int(np.sum(o.rows["lbin"][b] == l))
        want = 2.0 * m * ps[l, 0, 0] * d[b] / nm[l]
        assert abs(g - want) <= 1e-13 * max(abs(want), 1e-300)


def test_one_bin_bispectrum_pair(one_bin):
    """n_z = 1: B.B gives B_t B_t' / N(l) for every pair of legs in a common
    bin; the P.T part is P^s times the trispectrum of the remaining legs."""
    o = one_bin
    d, _ = o.data_vector()
    ps, nm = o.ps_table(), o.nmodes()
    B = np.where(o.rows["kind"] == 3)[0]
    for a in B:
        for b in B:
            la, lb = o.rows["lbin"][a], o.rows["lbin"][b]
            want = 0.0
            for x in range(3):
                for y in range(3):
                    if la[x] != lb[y]:
                        continue
                    rest = [la[q] for q in range(3) if q != x] + [lb[q] for q in range(3) if q != y]
                    want += (d[a] * d[b] + ps[la[x], 0, 0] * o.trispec(rest, [0, 0, 0, 0])) / nm[la[x]]
            got = o.ngins_pairs(np.array([[a, b]]))[0]
            assert abs(got - want) <= 1e-13 * max(abs(want), 1e-300)


def test_inverse_sky_fraction():
    """Every term carries 1 / N(l), N(l) proportional to f_sky."""
    t1 = synth.make_tables("tiny")
    t2 = dataclasses.replace(t1, cfg=dict(t1.cfg, f_sky=0.18))  # same tables
    o1, o2 = oracle.Oracle(t1), oracle.Oracle(t2)
    pairs = synth.sample_pairs(o1.N, 300, seed=9)
    v1, v2 = o1.ngins_pairs(pairs), o2.ngins_pairs(pairs)
    nz = v1 != 0
    assert np.count_nonzero(nz) > 20
    assert np.allclose(v2[nz] / v1[nz], t1.cfg["f_sky"] / t2.cfg["f_sky"], rtol=1e-13, atol=0)


def _bb_pb(o):
    """The B.B and P.B parts of the in-survey terms on all rows, from the
    projected bispectra, P^s and the mode counts (the remainder of the
    oracle's total is the P.T part)."""
    rows = o.rows
    kind, lb, zb, tri = rows["kind"], rows["lbin"], rows["zbin"], rows["tri"]
    Ps, nm, BF = o.ps_table(), o.nmodes(), o.bfull()
    N = o.N
    BB = np.zeros((N, N))
    PB = np.zeros((N, N))
    Bi = np.where(kind == 3)[0]
    Pi = np.where(kind == 2)[0]
    for a in Bi:
        for b in Bi:
            for x in range(3):
                for y in range(3):
                    if lb[a][x] != lb[b][y]:
                        continue
                    z1 = list(zb[a]); z2 = list(zb[b])
                    z1[x], z2[y] = zb[b][y], zb[a][x]
                    BB[a, b] += BF[tri[a], z1[0], z1[1], z1[2]] * BF[tri[b], z2[0], z2[1], z2[2]] / nm[lb[a][x]]
    for p in Pi:
        l, i, j = lb[p][0], zb[p][0], zb[p][1]
        for t in Bi:
            for y in range(3):
                if lb[t][y] != l:
                    continue
                zi = list(zb[t]); zj = list(zb[t])
                zi[y], zj[y] = i, j
                v = (Ps[l, zb[t][y], j] * BF[tri[t], zi[0], zi[1], zi[2]] +
                     Ps[l, i, zb[t][y]] * BF[tri[t], zj[0], zj[1], zj[2]]) / nm[l]
                PB[p, t] += v
                PB[t, p] += v
    return BB, PB


@pytest.mark.parametrize("n_z", [1, 2])
def test_term_structure(n_z):
    """P.T = P^s (x) T summed over shared modes is a Schur product of two
    positive semidefinite forms (P^s over the bins, the one-halo T a Gram
    over haloes), so it is positive semidefinite; B.B is a sum of
    u u^T / N(l) for one redshift bin and indefinite once it exchanges bins
    between the two rows; P.B only couples P and B rows."""
    o = oracle.Oracle(synth.make_tables("tiny", n_z=n_z))
    Cb = o.covariance()
    NG = o.covariance(ngins=True) - Cb
    BB, PB = _bb_pb(o)
    PT = NG - BB - PB
    s = 1.0 / np.sqrt(np.diag(Cb))
    scaled = lambda X: s[:, None] * X * s[None, :]
    assert np.linalg.eigvalsh(scaled(PT)).min() > -1e-12
    e_bb = np.linalg.eigvalsh(scaled(BB))
    if n_z == 1:
        assert e_bb.min() > -1e-12
    else:
        assert e_bb.min() < -1e-3 * e_bb.max()
    P = o.rows["kind"] == 2
    assert np.all(PB[np.ix_(P, P)] == 0.0) and np.all(PB[np.ix_(~P, ~P)] == 0.0)
    # the oracle's P-B block is exactly the P.B part (up to the rounding of the subtraction)
    assert np.max(np.abs(PT[np.ix_(P, ~P)])) <= 1e-12 * np.max(np.abs(PB))
