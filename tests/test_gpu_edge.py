"""Degenerate and boundary shapes through the whole C ABI against the
oracle: one redshift bin, one ell-bin (a single equilateral triangle),
and the smallest data vectors (N = 2), for the FP64 path, the chi
factorisation, the structured S/N, the ell_max curve and the PCA."""
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


@pytest.mark.parametrize("n_z,n_ell", [(1, 1), (1, 3), (4, 1), (3, 2)])
@pytest.mark.parametrize("precision", ["fp64", "fp64_chi"])
def test_degenerate_shapes(wl, n_z, n_ell, precision):
    _say("case edge n_z=%d n_ell=%d %s" % (n_z, n_ell, precision))
    t = synth.make_tables("tiny", n_z=n_z, n_ell=n_ell)
    o = oracle.Oracle(t)
    ref = o.run()
    prob = wl.Problem(t.cfg, t.arrays(), precision=precision)
    assert prob.sizes.n_data == o.N
    prob.run()
    snr2 = prob.snr2()
    torch.cuda.synchronize()
    assert np.max(np.abs(prob.d.cpu().numpy() - ref["d"]) / np.abs(ref["d"])) < 1e-10
    assert np.max(np.abs(prob.covariance_true() - ref["C"]) / np.abs(ref["C"])) < 1e-10
    assert abs(snr2 - ref["snr2"]) < 1e-10 * ref["snr2"]
    st = prob.snr2_structured()
    assert abs(st - ref["snr2"]) < 1e-10 * ref["snr2"]
    curve = prob.snr2_lmax()
    want = o.snr2_lmax(ref["C"], ref["d"])
    assert np.max(np.abs(curve - want) / want) < 1e-10
    lam, snr, cum, sweeps, S = prob.pca()
    lam0, snr0, cum0, _ = oracle.Oracle.pca(ref["C"], ref["d"])
    assert np.max(np.abs(lam / lam0 - 1.0)) < 1e-9
    assert np.max(np.abs(cum - cum0)) < 1e-9 * cum0[-1]
    prob.close()


@pytest.mark.parametrize("n_z,n_ell", [(1, 1), (1, 3), (4, 1), (3, 2)])
@pytest.mark.parametrize("precision", ["bf16_auto", "bf16x3"])
def test_degenerate_shapes_mixed(wl, n_z, n_ell, precision):
    """The bf16 products on the smallest shapes (one 256-row tile, mostly
    padding rows, one k-slice): the data vector stays FP64 (1e-10);
    covariance entries within 1e-5 of sqrt(C_aa C_bb) and (S/N)^2 within
    1e-4, the targets of the mixed-precision path."""
    _say("case edge mixed n_z=%d n_ell=%d %s" % (n_z, n_ell, precision))
    t = synth.make_tables("tiny", n_z=n_z, n_ell=n_ell)
    o = oracle.Oracle(t)
    ref = o.run()
    prob = wl.Problem(t.cfg, t.arrays(), precision=precision)
    assert prob.sizes.n_data == o.N
    prob.run()
    snr2 = prob.snr2()
    torch.cuda.synchronize()
    assert np.max(np.abs(prob.d.cpu().numpy() - ref["d"]) / np.abs(ref["d"])) < 1e-10
    dr = np.diag(ref["C"])
    err = np.max(np.abs(prob.covariance_true() - ref["C"]) / np.sqrt(np.outer(dr, dr)))
    _say("  C err %.2e, (S/N)^2 err %.2e" % (err, abs(snr2 - ref["snr2"]) / ref["snr2"]))
    assert err < 1e-5
    assert abs(snr2 - ref["snr2"]) < 1e-4 * ref["snr2"]
    st = prob.snr2_structured()
    assert abs(st - ref["snr2"]) < 1e-4 * ref["snr2"]
    curve = prob.snr2_lmax()
    want = o.snr2_lmax(ref["C"], ref["d"])
    assert np.max(np.abs(curve - want) / want) < 1e-4
    prob.close()
