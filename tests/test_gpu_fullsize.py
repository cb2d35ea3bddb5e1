"""Parity at the benchmark's full size, in the launch configuration bench.py
times: n_z = 10, 15 ell-bins over 10-5000, N_chi x N_M = 512 x 256
(K = 131072), N = 82575 data-vector rows, N_R = 33165 distinct rows.

The oracle evaluates the data vector and response entirely and the
covariance on seeded samples, one entry at a time.  The FP64 GPU path must
match it to 1e-10; the split-bf16 (bf16x3) path and the per-tile precision
the benchmark runs (bf16_auto: one bf16 product on every tile whose
a-priori bound is within 2^-17 of sqrt(C_aa C_bb), which at this size is
every tile) to 1e-5 on the diagonal and on off-diagonal entries relative to
sqrt(C_aa C_bb).  The oracle's Cholesky
cannot reach N = 82575, so the mixed-precision S/N is compared with the FP64
GPU path's, which the smaller workloads pin to the oracle."""
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


@pytest.fixture(scope="module")
def ref():
    t = synth.make_tables("large10")
    o = oracle.Oracle(t)
    _say("oracle data vector, N = %d" % o.N)
    d, r = o.data_vector()
    rng = np.random.default_rng(42)
    off = synth.sample_pairs(o.N, 300, seed=42)
    off = off[off[:, 0] != off[:, 1]]
    rows = np.unique(np.concatenate([off.ravel(), rng.integers(0, o.N, 200)]))
    diag = np.stack([rows, rows], 1)
    _say("oracle covariance: %d diagonal + %d off-diagonal entries" % (len(diag), len(off)))
    want_diag = dict(zip(rows.tolist(), o.cov_pairs(diag)))
    want_off = o.cov_pairs(off)
    return dict(t=t, N=o.N, d=d, r=r, rows=rows, want_diag=want_diag, off=off, want_off=want_off)


def _entries(prob, pairs):
    """C_true at the given (a, b) pairs, gathered on the device."""
    a = torch.as_tensor(pairs[:, 0], device=prob.C.device, dtype=torch.long)
    b = torch.as_tensor(pairs[:, 1], device=prob.C.device, dtype=torch.long)
    t = prob.row_exp2.long()
    v = prob.C[a, b].double() * torch.exp2(-(t[a] + t[b]).double())
    sym = bool(torch.equal(prob.C[a, b], prob.C[b, a]))
    return v.cpu().numpy(), sym


def _check(prob, ref, tol_diag, tol_off):
    assert np.max(np.abs(prob.d.cpu().numpy() - ref["d"]) / np.abs(ref["d"])) < 1e-10
    assert np.max(np.abs(prob.r.cpu().numpy() - ref["r"]) / np.abs(ref["r"])) < 1e-10
    rows = ref["rows"]
    got_d, _ = _entries(prob, np.stack([rows, rows], 1))
    want_d = np.array([ref["want_diag"][a] for a in rows.tolist()])
    err_d = np.max(np.abs(got_d - want_d) / want_d)
    got_o, sym = _entries(prob, ref["off"])
    scale = np.sqrt([ref["want_diag"][a] * ref["want_diag"][b] for a, b in ref["off"].tolist()])
    err_o = np.max(np.abs(got_o - ref["want_off"]) / scale)
    _say("  diag max rel %.3e, off-diag max rel to sqrt(C_aa C_bb) %.3e" % (err_d, err_o))
    assert sym
    assert err_d < tol_diag
    assert err_o < tol_off


def test_large10_fp64_chi_and_mixed(wl, ref):
    t = ref["t"]
    _say("case large10 fp64")
    p64 = wl.Problem(t.cfg, t.arrays(), precision="fp64")
    assert p64.sizes.n_data == 82575 and p64.sizes.n_distinct == 33165
    p64.run()
    snr64 = p64.snr2()
    torch.cuda.synchronize()
    _check(p64, ref, 1e-10, 1e-10)
    p64.close()
    del p64
    torch.cuda.empty_cache()

    _say("case large10 fp64_chi")
    pc = wl.Problem(t.cfg, t.arrays(), precision="fp64_chi")
    pc.run()
    snr_chi = pc.snr2()
    torch.cuda.synchronize()
    _check(pc, ref, 1e-10, 1e-10)
    _say("  (S/N)^2 fp64_chi %.12e fp64 %.12e" % (snr_chi, snr64))
    assert abs(snr_chi - snr64) / snr64 < 1e-9
    snr_st = pc.snr2_structured()
    _say("  (S/N)^2 structured (fp64_chi) %.12e" % snr_st)
    assert abs(snr_st - snr64) / snr64 < 1e-9
    pc.free_snr_workspace()
    pc.close()
    del pc
    torch.cuda.empty_cache()

    _say("case large10 bf16x3")
    pm = wl.Problem(t.cfg, t.arrays(), precision="bf16x3")
    pm.run()
    snr = pm.snr2()
    torch.cuda.synchronize()
    _check(pm, ref, 1e-5, 1e-5)
    _say("  (S/N)^2 bf16x3 %.9e fp64 %.9e" % (snr, snr64))
    assert abs(snr - snr64) / snr64 < 1e-4
    pm.free_snr_workspace()
    snr_st = pm.snr2_structured()
    _say("  (S/N)^2 structured (bf16x3) %.9e" % snr_st)
    assert abs(snr_st - snr64) / snr64 < 1e-4
    pm.close()
    del pm
    torch.cuda.empty_cache()

    _say("case large10 bf16_auto (the benchmark's precision)")
    pa = wl.Problem(t.cfg, t.arrays(), precision="bf16_auto")
    pa.run()
    snr = pa.snr2()
    torch.cuda.synchronize()
    split, tiles = pa.split_tiles()
    _say("  split tiles %d of %d" % (split, tiles))
    assert tiles == 130 * 131 // 2 and split == 0
    _check(pa, ref, 1e-5, 1e-5)
    _say("  (S/N)^2 bf16_auto %.9e fp64 %.9e" % (snr, snr64))
    assert abs(snr - snr64) / snr64 < 1e-4
    pa.close()
    del pa
    torch.cuda.empty_cache()


def test_large10_ngins_sampled(wl, ref):
    """The B.B, P.T and P.B terms at full size: sampled entries against the
    oracle (FP64, one-halo term factorised along chi)."""
    t = ref["t"]
    o = oracle.Oracle(t)
    pairs = np.concatenate([ref["off"][:200], np.stack([ref["rows"][:200]] * 2, 1)])
    _say("oracle with B.B, P.T, P.B terms: %d entries" % len(pairs))
    want = o.cov_pairs(pairs, ngins=True)
    _say("case large10 fp64_chi with the in-survey terms")
    pc = wl.Problem(t.cfg, t.arrays(), precision="fp64_chi", ngins=True)
    pc.run()
    torch.cuda.synchronize()
    got, sym = _entries(pc, pairs)
    assert sym
    scale = np.sqrt(np.abs(o.cov_pairs(np.stack([pairs[:, 0], pairs[:, 0]], 1), ngins=True) *
                           o.cov_pairs(np.stack([pairs[:, 1], pairs[:, 1]], 1), ngins=True)))
    err = np.max(np.abs(got - want) / scale)
    _say("  max rel to sqrt(C_aa C_bb) %.3e" % err)
    assert err < 1e-10
    pc.close()
    del pc
    torch.cuda.empty_cache()


def test_large10_ssc_chi_sampled(wl, ref):
    """The super-sample term resolved along chi at full size (FP64, one-halo
    term factorised along chi): sampled entries against the oracle, and the
    structured S/N against the plain one."""
    t = ref["t"]
    o = oracle.Oracle(t)
    pairs = np.concatenate([ref["off"][:200], np.stack([ref["rows"][:200]] * 2, 1)])
    _say("oracle with the chi-resolved super-sample term: %d entries" % len(pairs))
    want = o.cov_pairs(pairs, ssc="chi")
    _say("case large10 fp64_chi ssc_chi")
    pc = wl.Problem(t.cfg, t.arrays(), precision="fp64_chi", ssc_chi=True)
    pc.run()
    snr = pc.snr2()
    torch.cuda.synchronize()
    got, sym = _entries(pc, pairs)
    assert sym
    scale = np.sqrt(np.abs(o.cov_pairs(np.stack([pairs[:, 0], pairs[:, 0]], 1), ssc="chi") *
                           o.cov_pairs(np.stack([pairs[:, 1], pairs[:, 1]], 1), ssc="chi")))
    err = np.max(np.abs(got - want) / scale)
    _say("  max rel to sqrt(C_aa C_bb) %.3e" % err)
    assert err < 1e-10
    pc.free_snr_workspace()
    st = pc.snr2_structured()
    _say("  (S/N)^2 plain %.12e structured %.12e" % (snr, st))
    assert abs(st - snr) / snr < 1e-9
    pc.close()
    del pc
    torch.cuda.empty_cache()


def test_large10_snr2_lmax(wl, ref):
    """The ell_max curve at full size (bf16x3 covariance, FP64 Cholesky):
    increasing, and its last entry is the (S/N)^2 of wlc_snr2."""
    t = ref["t"]
    _say("case large10 bf16x3 snr2_lmax")
    pm = wl.Problem(t.cfg, t.arrays(), precision="bf16x3")
    pm.run()
    snr = pm.snr2()
    curve = pm.snr2_lmax()
    _say("  curve %s" % np.array2string(curve, precision=4))
    assert len(curve) == 15 and np.all(np.diff(curve) > 0)
    assert abs(curve[-1] - snr) / snr < 1e-6  # the same C factored in another row order
    pm.close()
    del pm
    torch.cuda.empty_cache()
