"""Parity of the HIP path (through the C ABI) with the FP64 oracle."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def wl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1812_07437_amd import wlcov
    return wlcov


_ORACLE = {}


def _oracle_full(preset, tomo="paper", ngins=False, **kw):
    key = (preset, tomo, ngins, tuple(sorted(kw.items())))
    if key not in _ORACLE:
        t = synth.make_tables(preset, **kw)
        o = oracle.Oracle(t, tomo=tomo)
        _ORACLE[key] = (t, o, o.run(ngins=ngins))
    return _ORACLE[key]


def _run(wl, t, precision="fp64", tomo="paper", snr=True, ngins=False):
    prob = wl.Problem(t.cfg, t.arrays(), precision=precision, tomo=tomo, ngins=ngins)
    prob.run()
    s = prob.snr2() if snr else None
    torch.cuda.synchronize()
    return prob, s


def _rel(a, b):
    return np.max(np.abs(a - b) / np.abs(b))


@pytest.mark.parametrize("precision", ["fp64", "fp64_chi"])
@pytest.mark.parametrize("preset,tomo", [("tiny", "paper"), ("tiny", "sorted"), ("mid", "paper")])
def test_fp64_full_parity(wl, preset, tomo, precision):
    """Both FP64 one-halo forms: the flattened Gram, and the sum over M
    first and chi second (factorisation along the line of sight)."""
    _say("case %s full %s %s" % (precision, preset, tomo))
    t, o, ref = _oracle_full(preset, tomo)
    prob, snr2 = _run(wl, t, precision, tomo)
    d = prob.d.cpu().numpy(); r = prob.r.cpu().numpy()
    assert _rel(d, ref["d"]) < 1e-10
    assert _rel(r, o.data_vector()[1]) < 1e-10
    C = prob.covariance_true()
    assert _rel(C, ref["C"]) < 1e-10
    Cs = prob.C.cpu().numpy()
    assert np.array_equal(Cs, Cs.T)
    dg = np.diag(Cs)
    assert np.all((dg >= 1.0) & (dg < 4.0))
    assert abs(snr2 - ref["snr2"]) / ref["snr2"] < 1e-10
    prob.close()


def test_fp64_deterministic(wl):
    _say("case fp64 determinism mid")
    t = synth.make_tables("mid")
    a, sa = _run(wl, t, "fp64")
    b, sb = _run(wl, t, "fp64")
    assert torch.equal(a.C, b.C) and torch.equal(a.d, b.d) and sa == sb


@pytest.mark.parametrize("precision", ["fp64", "fp64_chi"])
def test_fp64_euclid5_sampled(wl, precision):
    """Full-size 5-bin workload (N = 4550, K = 32768): data vector and response
    entirely, covariance on seeded samples including the diagonal."""
    _say("case %s euclid5 sampled" % precision)
    t = synth.make_tables("euclid5")
    o = oracle.Oracle(t)
    prob, _ = _run(wl, t, precision, snr=False)
    d_ref, r_ref = o.data_vector()
    assert _rel(prob.d.cpu().numpy(), d_ref) < 1e-10
    assert _rel(prob.r.cpu().numpy(), r_ref) < 1e-10
    pairs = np.concatenate([synth.sample_pairs(o.N, 1500, seed=42),
                            np.stack([np.arange(0, o.N, 7)] * 2, 1)])
    want = o.cov_pairs(pairs)
    C = prob.covariance_true()
    got = C[pairs[:, 0], pairs[:, 1]]
    assert _rel(got, want) < 1e-10
    Cs = prob.C
    assert torch.equal(Cs, Cs.T)
    prob.close()


@pytest.mark.parametrize("precision", ["bf16_auto", "bf16x3", "fp32"])
def test_mixed_precision_sorted(wl, precision):
    """SORTED tomography (N = N_R: the data vector is the distinct rows, the
    product's A-row order a permutation of the output's) with the
    mixed-precision targets: 1e-5 on the diagonal and on entries relative to
    sqrt(C_aa C_bb), 1e-4 on (S/N)^2."""
    for preset in ("tiny", "mid"):
        _say("case mixed sorted %s %s" % (precision, preset))
        t, o, ref = _oracle_full(preset, "sorted")
        prob, snr2 = _run(wl, t, precision, "sorted")
        C = prob.covariance_true()
        dr = np.diag(ref["C"])
        err_off = np.max(np.abs(C - ref["C"]) / np.sqrt(np.outer(dr, dr)))
        err_snr = abs(snr2 - ref["snr2"]) / ref["snr2"]
        _say("  %s sorted %s: C %.2e snr %.2e" % (precision, preset, err_off, err_snr))
        assert _rel(prob.d.cpu().numpy(), ref["d"]) < 1e-10
        assert err_off < 1e-5 and err_snr < 1e-4
        prob.close()


@pytest.mark.parametrize("precision,tol_diag,tol_off,tol_snr", [("bf16x3", 1e-5, 1e-5, 1e-4),
                                                                ("fp32", 1e-5, 1e-5, 1e-4),
                                                                ("bf16", 5e-3, 6e-3, 5e-2)])
def test_mixed_precision_tiny_mid(wl, precision, tol_diag, tol_off, tol_snr):
    """Tolerances: the diagonal and S/N targets of the mixed-precision path;
    off-diagonal entries relative to sqrt(C_aa C_bb), bounded by the relative
    error of one product term plus the FP32 accumulation (the derivation is
    in test_gpu_precision.py)."""
    for preset in ("tiny", "mid"):
        _say("case mixed %s %s" % (precision, preset))
        t, o, ref = _oracle_full(preset)
        prob, snr2 = _run(wl, t, precision)
        C = prob.covariance_true()
        dg = np.diag(C); dr = np.diag(ref["C"])
        err_diag = _rel(dg, dr)
        s = np.sqrt(np.outer(dr, dr))
        err_off = np.max(np.abs(C - ref["C"]) / s)
        err_snr = abs(snr2 - ref["snr2"]) / ref["snr2"]
        _say("  %s %s: diag %.2e offdiag/sqrt(CaaCbb) %.2e snr %.2e" % (precision, preset, err_diag, err_off,
                                                                      err_snr))
        assert err_diag < tol_diag
        assert err_off < tol_off
        assert err_snr < tol_snr
        assert _rel(prob.d.cpu().numpy(), ref["d"]) < 1e-10
        prob.close()


def test_validation_errors(wl):
    _say("case validation errors")
    t = synth.make_tables("tiny")
    arr = t.arrays()
    bad = dict(arr); P = arr["P"].copy(); P[3, 7] = np.nan; bad["P"] = P
    prob = wl.Problem(t.cfg, bad, "fp64")
    with pytest.raises(wl.WlcError) as e:
        prob.run()
    assert e.value.code == wl.WLC_EINVAL
    short = dict(arr)  # the table starts above ell_min / chi_max
    short["k"] = arr["k"] * (2.0 * t.cfg["ell_min"] / (t.chi[-1] * arr["k"][0]))
    prob = wl.Problem(t.cfg, short, "fp64")
    with pytest.raises(wl.WlcError) as e:
        prob.run()
    assert e.value.code == wl.WLC_ERANGE


def test_lattice_counts_bruteforce(wl):
    """Integer lattice counts bit-exact against pair-by-pair counting on a
    coarse lattice (small sky fraction) and on the first triangles of the
    tiny workload."""
    _say("case lattice coarse")
    t = synth.make_tables("tiny", f_sky=0.01)
    prob = wl.Problem(t.cfg, t.arrays(), "fp64")
    modes, tris = prob.lattice_counts()
    torch.cuda.synchronize()
    o = oracle.Oracle(t)
    thr = oracle.lattice_thresholds(o.edges, 0.01)
    assert [oracle.lattice_modes(thr, b) for b in range(o.n_ell)] == modes.cpu().tolist()
    want = [oracle.lattice_triangles(thr, i, j, k) for (i, j, k, _) in o.tris]
    assert tris.cpu().tolist() == want
    _say("case lattice tiny")
    t = synth.make_tables("tiny")
    prob = wl.Problem(t.cfg, t.arrays(), "fp64")
    modes, tris = prob.lattice_counts()
    torch.cuda.synchronize()
    o = oracle.Oracle(t)
    thr = oracle.lattice_thresholds(o.edges, t.cfg["f_sky"])
    assert [oracle.lattice_modes(thr, b) for b in range(o.n_ell)] == modes.cpu().tolist()
    for q, (i, j, k, _) in enumerate(o.tris[:4]):
        assert int(tris[q]) == oracle.lattice_triangles(thr, i, j, k)


@pytest.mark.parametrize("preset", ["tiny", "mid", "euclid5"])
def test_snr2_random_spd(wl, preset):
    """wlc_snr2 on a seeded random SPD matrix of the plan's size (several
    64-wide panels and a ragged last panel), against a LAPACK solve."""
    _say("case snr2 random spd %s" % preset)
    t = synth.make_tables(preset) if preset != "euclid5" else None
    cfg = t.cfg if t is not None else dict(synth.PRESETS["euclid5"], **synth.SURVEY_DEFAULTS, rho_mean=8.3e10)
    prob = wl.Problem(cfg, synth.make_tables("tiny").arrays(), precision="fp64")
    n = prob.sizes.n_data
    rng = np.random.default_rng(5)
    B = rng.standard_normal((n, n)) / np.sqrt(n)
    M = B @ B.T + 0.05 * np.eye(n)
    d = rng.standard_normal(n)
    e = rng.integers(-30, 30, n)
    Ms = np.ldexp(M, e[:, None] + e[None, :])
    prob.C.copy_(torch.from_numpy(Ms))
    prob.row_exp2.copy_(torch.from_numpy(e.astype(np.int32)))
    prob.d.copy_(torch.from_numpy(d))
    got = prob.snr2()
    want = float(d @ np.linalg.solve(M, d))
    assert abs(got - want) / want < 1e-9
    # not positive definite -> WLC_ENOTPD
    bad = Ms.copy()
    bad[n // 2, n // 2] = -1.0
    prob.C.copy_(torch.from_numpy(bad))
    with pytest.raises(wl.WlcError) as ex:
        prob.snr2()
    assert ex.value.code == wl.WLC_ENOTPD
    prob.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp64_chi", 1e-10), ("bf16x3", 1e-4)])
@pytest.mark.parametrize("preset", ["tiny", "mid"])
def test_snr2_structured(wl, preset, precision, tol):
    """(S/N)^2 through the distinct rows equals the oracle's d^T C^-1 d and
    the direct bordered Cholesky on the whole covariance."""
    _say("case structured snr2 %s %s" % (preset, precision))
    t, o, ref = _oracle_full(preset, "paper")
    prob, direct = _run(wl, t, precision, "paper")
    got = prob.snr2_structured()
    torch.cuda.synchronize()
    assert abs(got - ref["snr2"]) / ref["snr2"] < tol
    assert abs(got - direct) / direct < (1e-10 if precision != "bf16x3" else 1e-6)
    prob.close()


def test_snr2_structured_sorted_rejected(wl):
    _say("case structured snr2 sorted rejected")
    t = synth.make_tables("tiny")
    prob = wl.Problem(t.cfg, t.arrays(), precision="fp64", tomo="sorted")
    assert prob.sizes.ws_snr_structured_bytes == 0
    prob.run()
    with pytest.raises(wl.WlcError) as e:
        wl.wlc_snr2_structured(prob.plan, wl._ptr(prob.ws), wl._ptr(prob.ws), None)
    assert e.value.code == wl.WLC_EINVAL
    prob.close()


def test_snr2_structured_euclid5(wl):
    _say("case structured snr2 euclid5")
    t = synth.make_tables("euclid5")
    prob, direct = _run(wl, t, "fp64_chi")
    got = prob.snr2_structured()
    torch.cuda.synchronize()
    _say("  structured %.15e direct %.15e" % (got, direct))
    assert abs(got - direct) / direct < 1e-9
    prob.close()


@pytest.mark.parametrize("precision", ["fp64", "fp64_chi"])
@pytest.mark.parametrize("preset,tomo", [("tiny", "paper"), ("tiny", "sorted"), ("mid", "paper")])
def test_ngins_full_parity(wl, preset, tomo, precision):
    """With the B.B, P.T and P.B terms (eqs. CovBB, Covpb): the whole
    covariance and the S/N against the oracle."""
    _say("case ngins %s %s %s" % (precision, preset, tomo))
    t, o, ref = _oracle_full(preset, tomo, ngins=True)
    prob, snr2 = _run(wl, t, precision, tomo, ngins=True)
    C = prob.covariance_true()
    assert _rel(C, ref["C"]) < 1e-10
    Cs = prob.C.cpu().numpy()
    assert np.array_equal(Cs, Cs.T)
    dg = np.diag(Cs)
    assert np.all((dg >= 1.0) & (dg < 4.0))
    assert abs(snr2 - ref["snr2"]) / ref["snr2"] < 1e-10
    with pytest.raises(wl.WlcError):
        prob.snr2_structured()
    prob.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp64_chi", 1e-10), ("bf16x3", 1e-4)])
@pytest.mark.parametrize("preset,tomo", [("tiny", "paper"), ("tiny", "sorted"), ("mid", "paper")])
def test_snr2_lmax_curve(wl, preset, tomo, precision, tol):
    """(S/N)^2 at every ell_max cut from one Cholesky in ell_max order,
    against the oracle's curve (itself pinned to separately planned cut
    vectors)."""
    _say("case snr2_lmax %s %s %s" % (precision, preset, tomo))
    t, o, ref = _oracle_full(preset, tomo)
    want = o.snr2_lmax(ref["C"], ref["d"])
    prob, snr2 = _run(wl, t, precision, tomo)
    got = prob.snr2_lmax()
    assert got.shape == want.shape
    assert np.max(np.abs(got - want) / want) < tol
    assert abs(got[-1] - snr2) / snr2 < (1e-12 if precision != "bf16x3" else 1e-6)
    prob.close()
