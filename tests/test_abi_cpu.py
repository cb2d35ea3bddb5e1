"""Host-side checks of libwlcov: exported symbols, planning and counts against
the oracle's enumeration, argument validation.  No GPU needed."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

w = pytest.importorskip("paper_1812_07437_amd.wlcov", reason="libwlcov.so not built")


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?\s*(wlc_\w+)\s*\(", src, re.M))
    return names


def test_exports_every_declared_symbol():
    names = _declared_symbols()
    assert {"wlc_plan_create", "wlc_run", "wlc_snr2", "wlc_lattice_counts"} <= names
    lib = ct.CDLL(w.LIB_PATH)
    for n in sorted(names):
        assert hasattr(lib, n), n
    for n in w.EXPORTED:
        assert n in names


def _plan(preset, tomo="paper", **over):
    t = dict(synth.PRESETS[preset]) if isinstance(preset, str) else dict(preset)
    t.update(synth.SURVEY_DEFAULTS)
    t["rho_mean"] = 0.3 * synth.RHO_CRIT
    t.update(over)
    cfg = w.make_config(t, "fp64", tomo)
    return t, w.wlc_plan_create(cfg)


def _index(plan):
    s = w.wlc_plan_sizes(plan)
    tri = np.zeros((max(1, s.n_tri), 3), np.int32)
    rows = np.zeros((s.n_data, 8), np.int32)
    dist = np.zeros(s.n_data, np.int32)
    w.wlc_plan_index(plan, tri.ctypes.data_as(ct.c_void_p), rows.ctypes.data_as(ct.c_void_p),
                     dist.ctypes.data_as(ct.c_void_p))
    return s, tri[:s.n_tri], rows, dist


@pytest.mark.parametrize("preset,tomo", [("tiny", "paper"), ("tiny", "sorted"), ("mid", "paper"),
                                         ("euclid5", "paper"), ("large10", "paper"), ("large10", "sorted")])
def test_enumeration_bit_exact_vs_oracle(preset, tomo):
    t, plan = _plan(preset, tomo)
    s, tri, rows, dist = _index(plan)
    _, cen, _ = oracle.ell_bins(t["ell_min"], t["ell_max"], t["n_ell"])
    ref = oracle.enumerate_rows(t["n_z"], t["n_ell"], cen, tomo)
    assert s.n_data == len(ref["kind"])
    assert np.array_equal(tri, np.array([x[:3] for x in ref["triangles"]], np.int32).reshape(-1, 3))
    assert np.array_equal(rows[:, 0], ref["kind"])
    assert np.array_equal(rows[:, 1], ref["cfg"])
    lb = ref["lbin"].copy()
    lb[ref["kind"] == 2, 1] = lb[ref["kind"] == 2, 0]
    assert np.array_equal(rows[:, 2:5], lb)
    assert np.array_equal(rows[:, 5:8], ref["zbin"])
    # distinct map: same class iff same canonical key, and the distinct
    # vector is the sorted-tomography vector
    canon, reps = oracle.canonical_rows(ref)
    assert s.n_distinct == len(reps)
    pairs = {}
    for a, (c, e) in enumerate(zip(canon, dist)):
        assert pairs.setdefault(int(c), int(e)) == int(e)
    assert len(set(dist.tolist())) == len(reps)
    w.wlc_plan_destroy(plan)


def test_closed_counts_vs_oracle():
    t, plan = _plan("euclid5")
    s = w.wlc_plan_sizes(plan)
    nm = np.zeros(s.n_ell_used); nt = np.zeros(s.n_tri)
    w.wlc_counts_closed(plan, nm.ctypes.data_as(ct.c_void_p), nt.ctypes.data_as(ct.c_void_p))
    _, cen, wid = oracle.ell_bins(t["ell_min"], t["ell_max"], t["n_ell"])
    assert np.allclose(nm, oracle.n_modes(cen, wid, t["f_sky"]), rtol=1e-14)
    want = [oracle.n_tri_closed(cen[i], cen[j], cen[k], wid[i], wid[j], wid[k], t["f_sky"])
            for (i, j, k, _) in oracle.triangles(cen)]
    # Lambda^2 cancels for near-flat triangles: allow the amplified rounding
    assert np.allclose(nt, want, rtol=1e-11)
    w.wlc_plan_destroy(plan)


def test_ell_cut_plan():
    t, plan = _plan("large10", ell_cut=1000.0)
    s = w.wlc_plan_sizes(plan)
    assert s.n_ell_used == 11
    _, cen, _ = oracle.ell_bins(10.0, 5000.0, 15)
    ref = oracle.enumerate_rows(10, 11, cen)
    assert s.n_data == len(ref["kind"])
    w.wlc_plan_destroy(plan)


@pytest.mark.parametrize("bad", [dict(n_z=0), dict(ell_min=-1.0), dict(f_sky=1.5), dict(k_max=0.0),
                                 dict(ell_cut=5.0), dict(n_k=1)])
def test_invalid_config_rejected(bad):
    t = dict(synth.PRESETS["tiny"]); t.update(synth.SURVEY_DEFAULTS); t["rho_mean"] = 1e11
    t.update(bad)
    cfg = w.make_config(t)
    with pytest.raises(w.WlcError) as e:
        w.wlc_plan_create(cfg)
    assert e.value.code == w.WLC_EINVAL
    assert w.wlc_last_error()


@pytest.mark.parametrize("preset,tomo", [("mid", "paper"), ("euclid5", "paper"), ("euclid5", "sorted")])
def test_gram_order(preset, tomo):
    """The flattened products take the distinct rows stably by their lowest
    redshift bin (a permutation); the chi-factorised one keeps the distinct
    order."""
    t = dict(synth.PRESETS[preset]); t.update(synth.SURVEY_DEFAULTS); t["rho_mean"] = 0.3 * synth.RHO_CRIT
    for prec in ("bf16", "bf16x3", "bf16_auto", "fp32", "fp64", "fp64_chi"):
        plan = w.wlc_plan_create(w.make_config(t, prec, tomo))
        s, _, rows, dist = _index(plan)
        pos = np.zeros(s.n_distinct, np.int32)
        w.wlc_plan_gram_order(plan, pos.ctypes.data_as(ct.c_void_p))
        w.wlc_plan_destroy(plan)
        ident = np.arange(s.n_distinct)
        if prec == "fp64_chi":
            assert np.array_equal(pos, ident)
            continue
        assert np.array_equal(np.sort(pos), ident)
        z = rows[:, 5:8].astype(np.int64)
        low = np.full(s.n_distinct, -1, np.int64)
        low[dist] = np.where(z >= 0, z, 1 << 30).min(1)  # every data row of a distinct row has its bins
        assert (low >= 0).all()
        order = np.argsort(pos)  # distinct rows in product order
        assert np.array_equal(order, np.lexsort((ident, low)))


def test_precision_modes():
    t = dict(synth.PRESETS["tiny"]); t.update(synth.SURVEY_DEFAULTS); t["rho_mean"] = 1e11
    for name, code in w.PRECISIONS.items():
        plan = w.wlc_plan_create(w.make_config(t, name))
        s = w.wlc_plan_sizes(plan)
        assert s.c_elem_bytes == (8 if name in ("fp64", "fp64_chi") else 4)
        w.wlc_plan_destroy(plan)
    for bad in (6, -1):
        with pytest.raises(w.WlcError) as e:
            w.wlc_plan_create(w.make_config(t, bad))
        assert e.value.code == w.WLC_EINVAL


def test_null_arguments_rejected():
    _, plan = _plan("tiny")
    tabs = w.wlc_tables()
    with pytest.raises(w.WlcError) as e:
        w.wlc_run(plan, tabs, None, None, None, None, None, None)
    assert e.value.code == w.WLC_EINVAL
    with pytest.raises(w.WlcError):
        w.wlc_snr2(plan, None, None, None, None, None)
    w.wlc_plan_destroy(plan)


def test_workspace_sizes_cover_buffers():
    for prec, el in (("fp64", 8), ("bf16x3", 4)):
        t = dict(synth.PRESETS["large10"]); t.update(synth.SURVEY_DEFAULTS); t["rho_mean"] = 1e11
        p = w.wlc_plan_create(w.make_config(t, prec))
        s = w.wlc_plan_sizes(p)
        assert s.c_elem_bytes == el
        r_pad = -(-s.n_distinct // 128) * 128
        a_bytes = r_pad * s.k_len * (8 if prec == "fp64" else 4)
        assert s.ws_run_bytes > a_bytes + r_pad * r_pad * el
        assert s.ws_snr_bytes >= (s.n_data + 1) ** 2 * 8
        w.wlc_plan_destroy(p)


def test_chi_resolved_ssc_sizes():
    """With the line-of-sight super-sample term the Gram product gains one
    column per chi node; the rest of the plan is unchanged."""
    t = dict(synth.PRESETS["large10"]); t.update(synth.SURVEY_DEFAULTS); t["rho_mean"] = 1e11
    for prec in ("fp64", "bf16x3", "fp64_chi"):
        p0 = w.wlc_plan_create(w.make_config(t, prec))
        p1 = w.wlc_plan_create(w.make_config(t, prec, ssc_chi=True))
        s0, s1 = w.wlc_plan_sizes(p0), w.wlc_plan_sizes(p1)
        assert s0.k_len == t["n_chi"] * t["n_m"]
        assert s1.k_len == t["n_chi"] * (t["n_m"] + 1)
        assert (s1.n_data, s1.n_distinct, s1.ws_snr_bytes) == (s0.n_data, s0.n_distinct, s0.ws_snr_bytes)
        assert s1.ws_run_bytes > s0.ws_run_bytes
        w.wlc_plan_destroy(p0)
        w.wlc_plan_destroy(p1)
    _, plan = _plan("tiny")
    with pytest.raises(w.WlcError) as e:
        w.wlc_sigma_w2(plan, w.wlc_tables(), None, None)
    assert e.value.code == w.WLC_EINVAL
    w.wlc_plan_destroy(plan)


@pytest.mark.parametrize("preset,S", [("tiny", 1), ("tiny", 2), ("tiny", 3), ("mid", 2), ("large10", 3)])
def test_averaging_lists_vs_oracle(preset, S):
    """The plan's bin-averaging lists: the same entries (bit-exact legs) as
    the oracle's, weights to 1e-13 (Gauss-Legendre nodes computed
    independently on both sides)."""
    t = dict(synth.PRESETS[preset]); t.update(synth.SURVEY_DEFAULTS); t["rho_mean"] = 1e11
    plan = w.wlc_plan_create(w.make_config(t, "fp64", n_sub=S))
    s = w.wlc_plan_sizes(plan)
    off = np.zeros(s.n_cfg + 1, np.int32)
    legs = np.zeros((s.n_avg, 3), np.int32)
    ell = np.zeros(s.n_ell_used * S, np.float64)
    wt = np.zeros(s.n_avg, np.float64)
    w.wlc_plan_averaging(plan, *(a.ctypes.data_as(ct.c_void_p) for a in (off, legs, ell, wt)))
    w.wlc_plan_destroy(plan)
    edges, centres, widths = oracle.ell_bins(t["ell_min"], t["ell_max"], t["n_ell"])
    sub = oracle.sub_bin_centres(edges, centres, t["n_ell"], S)
    tris = oracle.triangles(centres)
    cl = [(b, b, -1) for b in range(t["n_ell"])] + [q[:3] for q in tris]
    ref = oracle.averaging_lists([2] * t["n_ell"] + [3] * len(tris), cl, S, sub, widths)
    assert np.allclose(ell, sub, rtol=1e-15, atol=0)
    assert off[-1] == s.n_avg == sum(len(W) for _, W in ref)
    for c, (L, W) in enumerate(ref):
        mine = legs[off[c]:off[c + 1]]
        if c < t["n_ell"]:
            assert np.array_equal(mine[:, :2], L[:, :2]) and np.all(mine[:, 2] == -1)
        else:
            assert np.array_equal(mine, L)
        assert np.allclose(wt[off[c]:off[c + 1]], W, rtol=1e-13, atol=0)


def test_averaging_arguments():
    t = dict(synth.PRESETS["tiny"]); t.update(synth.SURVEY_DEFAULTS); t["rho_mean"] = 1e11
    for bad in (dict(n_sub=9), dict(n_sub=-1), dict(n_sub=2, ngins=True)):
        with pytest.raises(w.WlcError) as e:
            w.wlc_plan_create(w.make_config(t, "fp64", **bad))
        assert e.value.code == w.WLC_EINVAL


def test_gram_arguments_rejected():
    """wlc_gram checks its arguments before anything touches the device (the
    pointers below are never dereferenced: every case fails a check first)."""
    assert w.wlc_gram_ws_bytes("bf16", 256, 64) == 0
    # one k-slice from about 2000 tiles on, for every bf16 mode
    assert w.wlc_gram_ws_bytes("bf16", 33165, 131072) == 0
    assert w.wlc_gram_ws_bytes("bf16x3", 33165, 131072) == 0
    # 55 tiles of the Euclid-like shape: four slices
    assert w.wlc_gram_ws_bytes("bf16", 2390, 32768) == 3 * 2560 * 2560 * 4
    assert w.wlc_gram_ws_bytes("bf16x3", 2390, 32768) == 3 * 2560 * 2560 * 4
    fake = 4096  # a non-null, 256-byte-aligned stand-in
    bad = [
        dict(precision="fp64"), dict(precision="fp32"), dict(n=0), dict(k=0), dict(n=(1 << 20) + 1),
        dict(a_hi=None), dict(g=None),
        dict(precision="bf16x3", a_lo=None), dict(precision="bf16_auto", a_lo=None),
        dict(precision="bf16_auto", panel_f=None),
        dict(n=256, k=4096, ws=None), dict(n=256, k=4096, ws=fake + 1),
    ]
    for b in bad:
        a = dict(precision="bf16", n=256, k=4096, a_hi=fake, a_lo=fake, panel_f=fake, lim=0.5, g=fake, ws=fake)
        a.update(b)
        with pytest.raises(w.WlcError) as e:
            w.wlc_gram(a["precision"], a["n"], a["k"], a["a_hi"], a["a_lo"], a["panel_f"], a["lim"], a["g"], a["ws"],
                       None)
        assert e.value.code == w.WLC_EINVAL, b
    with pytest.raises(w.WlcError):
        w.wlc_gram_ws_bytes("bf16", 0, 64)
