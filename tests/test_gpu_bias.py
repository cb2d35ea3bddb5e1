"""Parity with mass-dependent halo biases b1(M), b2(M) (eqs. ImunuHalos,
ImunuHalosDeltaB, PowerHMResp, BispHMResp): the bias tables change the data
vector (two- and three-halo terms carry I_1^1 and I_2^1), the responses
(I_2^1, I_2^2, I_3^1) and through them the super-sample term."""
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


def _ref(preset):
    if preset not in _REF:
        t = synth.with_bias(synth.make_tables(preset))
        o = oracle.Oracle(t)
        ref = o.run()
        r_ref = o.data_vector()[1]
        r_unbiased = oracle.Oracle(synth.make_tables(preset)).data_vector()[1]
        _REF[preset] = (t, ref, r_ref, r_unbiased)
    return _REF[preset]


def _rel(a, b):
    return np.max(np.abs(a - b) / np.abs(b))


@pytest.mark.parametrize("precision", ["fp64", "fp64_chi"])
@pytest.mark.parametrize("preset", ["tiny", "mid"])
def test_bias_fp64_parity(wl, preset, precision):
    _say("case bias %s %s" % (precision, preset))
    t, ref, r_ref, r_unb = _ref(preset)
    # the bias tables must matter for this test to mean anything
    assert _rel(r_ref, r_unb) > 1e-2
    prob = wl.Problem(t.cfg, t.arrays(), precision=precision)
    prob.run()
    snr2 = prob.snr2()
    torch.cuda.synchronize()
    assert _rel(prob.d.cpu().numpy(), ref["d"]) < 1e-10
    assert _rel(prob.r.cpu().numpy(), r_ref) < 1e-10
    assert _rel(prob.covariance_true(), ref["C"]) < 1e-10
    assert abs(snr2 - ref["snr2"]) / ref["snr2"] < 1e-10
    prob.close()


@pytest.mark.parametrize("preset", ["tiny", "mid"])
def test_bias_bf16x3(wl, preset):
    _say("case bias bf16x3 %s" % preset)
    t, ref, r_ref, _ = _ref(preset)
    prob = wl.Problem(t.cfg, t.arrays(), precision="bf16x3")
    prob.run()
    snr2 = prob.snr2()
    torch.cuda.synchronize()
    C = prob.covariance_true()
    assert _rel(np.diag(C), np.diag(ref["C"])) < 1e-5
    assert abs(snr2 - ref["snr2"]) / ref["snr2"] < 1e-4
    assert _rel(prob.r.cpu().numpy(), r_ref) < 1e-10
    prob.close()
