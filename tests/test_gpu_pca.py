"""Parity of the principal component analysis (Sec. 6) between the HIP path
(one-sided block Jacobi on FP64 MFMA, through the C ABI) and the oracle
(LAPACK's Jacobi SVD), on the same covariance definitions."""
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


_REF = {}


def _ref(preset, tomo):
    if (preset, tomo) not in _REF:
        t = synth.make_tables(preset)
        o = oracle.Oracle(t, tomo=tomo)
        r = o.run()
        _REF[(preset, tomo)] = (t, r, oracle.Oracle.pca(r["C"], r["d"]))
    return _REF[(preset, tomo)]


@pytest.mark.parametrize("precision", ["fp64", "fp64_chi"])
@pytest.mark.parametrize("preset,tomo", [("tiny", "paper"), ("tiny", "sorted"), ("mid", "paper")])
def test_pca_parity(wl, preset, tomo, precision):
    """Eigenvalues over all decades to 1e-9 relative, the cumulative curve to
    1e-9 of the total, and the eigenvectors of well-separated modes."""
    _say("case pca %s %s %s" % (precision, preset, tomo))
    t, r, (lam0, snr0, cum0, S0) = _ref(preset, tomo)
    prob = wl.Problem(t.cfg, t.arrays(), precision=precision, tomo=tomo)
    prob.run()
    snr2 = prob.snr2()
    lam, snr, cum, sweeps, S = prob.pca()
    torch.cuda.synchronize()
    _say("  sweeps %d, lambda %.3e .. %.3e" % (sweeps, lam[0], lam[-1]))
    err = np.max(np.abs(lam / lam0 - 1.0))
    _say("  lambda max rel %.3e" % err)
    assert err < 1e-9
    assert np.max(np.abs(cum - cum0)) < 1e-9 * cum0[-1]
    assert abs(cum[-1] - snr2) < 1e-10 * snr2
    # modes whose eigenvalue is separated from its neighbours by > 1e-3
    gap = np.minimum(np.r_[np.inf, lam0[1:] / lam0[:-1] - 1], np.r_[lam0[1:] / lam0[:-1] - 1, np.inf])
    sep = gap > 1e-3
    assert np.count_nonzero(sep) > 0.5 * len(lam0)
    assert np.max(np.abs(snr[sep] - snr0[sep])) < 1e-8 * cum0[-1]
    Sg = S.cpu().numpy()
    assert np.max(np.abs(Sg[sep] - S0[sep])) < 1e-7
    prob.close()


def test_pca_mixed(wl):
    """bf16x3 covariance: the cumulative curve within 1e-4 of the FP64 one."""
    _say("case pca bf16x3 mid")
    t, r, (lam0, snr0, cum0, S0) = _ref("mid", "paper")
    prob = wl.Problem(t.cfg, t.arrays(), precision="bf16x3")
    prob.run()
    lam, snr, cum, sweeps, _ = prob.pca(vectors=False)
    assert np.max(np.abs(cum - cum0)) < 1e-4 * cum0[-1]
    prob.close()


def test_pca_euclid5_properties(wl):
    """Euclid-like size (N = 4550): the sum rule against the Cholesky S/N,
    ascending positive eigenvalues, orthonormal eigenvectors, and the
    reconstruction of sampled covariance entries."""
    _say("case pca fp64 euclid5")
    t = synth.make_tables("euclid5")
    prob = wl.Problem(t.cfg, t.arrays(), precision="fp64")
    prob.run()
    snr2 = prob.snr2()
    lam, snr, cum, sweeps, S = prob.pca()
    torch.cuda.synchronize()
    _say("  sweeps %d, lambda %.3e .. %.3e, (S/N)^2 %.6e vs %.6e" % (sweeps, lam[0], lam[-1], cum[-1], snr2))
    assert abs(cum[-1] - snr2) < 1e-9 * snr2
    assert np.all(lam > 0) and np.all(np.diff(lam) >= 0)
    G = S @ S.T
    assert torch.max(torch.abs(G - torch.eye(len(lam), dtype=G.dtype, device=G.device))).item() < 1e-10
    pairs = synth.sample_pairs(len(lam), 200, seed=3)
    a = torch.as_tensor(pairs[:, 0], device=S.device)
    b = torch.as_tensor(pairs[:, 1], device=S.device)
    L = torch.as_tensor(lam, device=S.device)
    rec = torch.sum(S[:, a] * S[:, b] * L[:, None], dim=0)
    te = prob.row_exp2.long()
    Ct = prob.C[a, b].double() * torch.exp2(-(te[a] + te[b]).double())
    sc = torch.sqrt(prob.C[a, a].double() * torch.exp2(-2.0 * te[a].double()) *
                    prob.C[b, b].double() * torch.exp2(-2.0 * te[b].double()))
    assert torch.max(torch.abs(rec - Ct) / sc).item() < 1e-9
    prob.close()


@pytest.mark.parametrize("n_z", [1, 2])
def test_pca_paper_binning(wl, n_z):
    """The paper's 14 ell-bins over 10-5000 with one and two redshift bins
    (N = 144 and 818): eigenvalues against the oracle, and the number of
    modes holding 99 % of (S/N)^2 the same on both sides unless the oracle's
    own cumulative curve sits within 1e-8 of that threshold."""
    _say("case pca paper binning n_z=%d" % n_z)
    t = synth.make_tables("paper14", n_z=n_z)
    r = oracle.Oracle(t).run()
    lam0, snr0, cum0 = oracle.Oracle.pca(r["C"], r["d"], vectors=False)
    prob = wl.Problem(t.cfg, t.arrays(), precision="fp64")
    prob.run()
    lam, snr, cum, sweeps, _ = prob.pca(vectors=False)
    torch.cuda.synchronize()
    err = np.max(np.abs(lam / lam0 - 1.0))
    _say("  N %d, sweeps %d, lambda max rel %.3e" % (len(lam), sweeps, err))
    assert len(lam) == {1: 144, 2: 818}[n_z]
    assert err < 1e-9
    assert np.max(np.abs(cum - cum0)) < 1e-9 * cum0[-1]
    thr = 0.99 * cum0[-1]
    k0 = int(np.searchsorted(cum0, thr) + 1)
    k = int(np.searchsorted(cum, 0.99 * cum[-1]) + 1)
    near = np.min(np.abs(cum0[max(0, k0 - 2):k0 + 1] - thr)) < 1e-8 * cum0[-1]
    assert k == k0 or near
    prob.close()
