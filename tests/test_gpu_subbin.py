"""Parity of bin averaging (n_sub sub-bins per ell-bin) between the HIP path
(through the C ABI) and the FP64 oracle: data vector, responses, covariance
and S/N, in every precision mode."""
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


def _rel(a, b):
    return np.max(np.abs(a - b) / np.abs(b))


_ORACLE = {}


def _oracle(preset, tomo, S, ssc="rank1"):
    key = (preset, tomo, S, ssc)
    if key not in _ORACLE:
        t = synth.make_tables(preset)
        o = oracle.Oracle(t, tomo=tomo, n_sub=S)
        _ORACLE[key] = (t, o, o.run(ssc=ssc))
    return _ORACLE[key]


@pytest.mark.parametrize("precision", ["fp64", "fp64_chi"])
@pytest.mark.parametrize("preset,tomo,S", [("tiny", "paper", 2), ("tiny", "paper", 3), ("tiny", "sorted", 2),
                                           ("mid", "paper", 2)])
def test_subbin_full_parity(wl, preset, tomo, S, precision):
    _say("case subbin %s %s %s n_sub=%d" % (precision, preset, tomo, S))
    t, o, ref = _oracle(preset, tomo, S)
    prob = wl.Problem(t.cfg, t.arrays(), precision=precision, tomo=tomo, n_sub=S)
    prob.run()
    snr2 = prob.snr2()
    torch.cuda.synchronize()
    assert _rel(prob.d.cpu().numpy(), ref["d"]) < 1e-10
    assert _rel(prob.r.cpu().numpy(), ref["r"]) < 1e-10
    C = prob.covariance_true()
    err = _rel(C, ref["C"])
    _say("  C max rel %.3e" % err)
    assert err < 1e-10
    Cs = prob.C.cpu().numpy()
    assert np.array_equal(Cs, Cs.T)
    assert abs(snr2 - ref["snr2"]) / ref["snr2"] < 1e-10
    if tomo == "paper":
        st = prob.snr2_structured()
        assert abs(st - ref["snr2"]) / ref["snr2"] < 1e-10
    prob.close()


def test_subbin_with_chi_resolved_ssc(wl):
    _say("case subbin + ssc_chi fp64 tiny n_sub=2")
    t, o, ref = _oracle("tiny", "paper", 2, ssc="chi")
    prob = wl.Problem(t.cfg, t.arrays(), precision="fp64", n_sub=2, ssc_chi=True)
    prob.run()
    snr2 = prob.snr2()
    torch.cuda.synchronize()
    assert _rel(prob.covariance_true(), ref["C"]) < 1e-10
    assert abs(snr2 - ref["snr2"]) / ref["snr2"] < 1e-10
    prob.close()


def test_subbin_mixed(wl):
    _say("case subbin bf16x3 tiny n_sub=3")
    t, o, ref = _oracle("tiny", "paper", 3)
    prob = wl.Problem(t.cfg, t.arrays(), precision="bf16x3", n_sub=3)
    prob.run()
    snr2 = prob.snr2()
    torch.cuda.synchronize()
    C = prob.covariance_true()
    dg = np.diag(ref["C"])
    assert np.max(np.abs(np.diag(C) - dg) / dg) < 1e-5
    assert np.max(np.abs(C - ref["C"]) / np.sqrt(np.outer(dg, dg))) < 1e-5
    assert abs(snr2 - ref["snr2"]) / ref["snr2"] < 1e-4
    prob.close()


def test_subbin_euclid5_sampled(wl):
    """Euclid-like size, two sub-bins per side: data vector in full, sampled
    covariance entries against the oracle."""
    _say("case subbin fp64_chi euclid5 n_sub=2 (oracle)")
    t = synth.make_tables("euclid5")
    o = oracle.Oracle(t, n_sub=2)
    d, r = o.data_vector()
    pairs = synth.sample_pairs(o.N, 300, seed=11)
    pairs = np.concatenate([pairs, np.stack([pairs[:50, 0]] * 2, 1)])
    want = o.cov_pairs(pairs)
    _say("case subbin fp64_chi euclid5 n_sub=2 (GPU)")
    prob = wl.Problem(t.cfg, t.arrays(), precision="fp64_chi", n_sub=2)
    prob.run()
    torch.cuda.synchronize()
    assert _rel(prob.d.cpu().numpy(), d) < 1e-10
    assert _rel(prob.r.cpu().numpy(), r) < 1e-10
    C = prob.C
    a = torch.as_tensor(pairs[:, 0], device=C.device)
    b = torch.as_tensor(pairs[:, 1], device=C.device)
    te = prob.row_exp2.long()
    got = (C[a, b].double() * torch.exp2(-(te[a] + te[b]).double())).cpu().numpy()
    dg = o.cov_pairs(np.stack([pairs[:, 0], pairs[:, 0]], 1)) * o.cov_pairs(np.stack([pairs[:, 1], pairs[:, 1]], 1))
    err = np.max(np.abs(got - want) / np.sqrt(dg))
    _say("  max rel to sqrt(C_aa C_bb) %.3e" % err)
    assert err < 1e-10
    prob.close()
