"""wlc_snr2_noalloc: the S/N of wlc_snr2 with the library's fixed device
scratch instead of a caller workspace, for callers that cannot allocate.
Checked through the C ABI against wlc_snr2 on two calls in a row (the
second with a smaller data vector), in FP64 and with an FP32 covariance."""
import math
import sys

import numpy as np
import pytest

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


def _noalloc(prob):
    out = torch.full((1,), math.nan, dtype=torch.float64, device="cuda:0")
    status = torch.full((1,), -7, dtype=torch.int32, device="cuda:0")
    prob.snr2_noalloc(out, status)
    torch.cuda.synchronize()
    return float(out.item()), int(status.item())


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_noalloc_matches_snr2_twice(wl, precision):
    for preset in ("mid", "tiny"):  # the second call has the smaller data vector
        _say("case noalloc %s %s" % (precision, preset))
        t = synth.make_tables(preset)
        prob = wl.Problem(t.cfg, t.arrays(), precision=precision)
        prob.run()
        want = prob.snr2()
        got, status = _noalloc(prob)
        _say("  N=%d snr2 %.17e vs %.17e" % (prob.sizes.n_data, got, want))
        assert status == 0
        assert abs(got - want) / want < 1e-10
        assert got == want  # same kernels and split choices
        prob.close()


def test_noalloc_not_positive_definite(wl):
    _say("case noalloc not positive definite")
    t = synth.make_tables("tiny")
    prob = wl.Problem(t.cfg, t.arrays(), precision="fp64")
    prob.run()
    n = prob.sizes.n_data
    prob.C[n // 2, n // 2] = -1.0  # set from the host: a negative pivot
    _, status = _noalloc(prob)
    assert status != 0
    with pytest.raises(wl.WlcError) as e:
        prob.snr2()
    assert e.value.code == wl.WLC_ENOTPD
    prob.close()


def test_noalloc_refuses_long_vectors(wl):
    """euclid5 (N = 4550) needs more than the 64 MiB scratch: refused before
    anything is enqueued."""
    _say("case noalloc refuses euclid5")
    cfg = dict(synth.PRESETS["euclid5"], **synth.SURVEY_DEFAULTS, rho_mean=8.3e10)
    plan = wl.wlc_plan_create(wl.make_config(cfg, "fp64"))
    dummy = torch.zeros(16, dtype=torch.float64, device="cuda:0")
    st = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    with pytest.raises(wl.WlcError) as e:
        wl.wlc_snr2_noalloc(plan, wl._ptr(dummy), wl._ptr(st), wl._ptr(dummy), wl._ptr(dummy), wl._ptr(st), None)
    assert e.value.code == wl.WLC_EINVAL
    wl.wlc_plan_destroy(plan)
    torch.cuda.synchronize()
    assert torch.count_nonzero(dummy).item() == 0
