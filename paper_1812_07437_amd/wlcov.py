"""ctypes binding of libwlcov (include/wlcov.h), with the same entry-point names.

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch provides device memory and streams.  Importing this module
fails loudly when the built library is missing.
"""
from __future__ import annotations

import ctypes as ct
import os

# torch ships its own HIP runtime with the same soname as the system one;
# loading it first makes libwlcov bind to that single runtime, which owns
# the device memory of every tensor passed in.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwlcov.so")

WLC_OK, WLC_EINVAL, WLC_ERANGE, WLC_ENOMEM, WLC_ENOTPD, WLC_EDEVICE, WLC_EBUSY, WLC_ENOCONV = 0, -1, -2, -3, -4, -5, -6, -7
WLC_TOMO_PAPER, WLC_TOMO_SORTED = 0, 1
WLC_FP64, WLC_BF16, WLC_BF16X3, WLC_FP32, WLC_FP64_CHI, WLC_BF16_AUTO = 0, 1, 2, 3, 4, 5
WLC_FLAG_NOCHECK, WLC_FLAG_NGINS, WLC_FLAG_SSC_CHI = 1, 2, 4
PRECISIONS = {"fp64": WLC_FP64, "bf16": WLC_BF16, "bf16x3": WLC_BF16X3, "fp32": WLC_FP32,
              "fp64_chi": WLC_FP64_CHI, "bf16_auto": WLC_BF16_AUTO}


def _prec(precision):
    """A precision code from its name or the code itself."""
    return PRECISIONS[precision] if isinstance(precision, str) else int(precision)


class WlcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("wlcov error %d: %s" % (code, msg))
        self.code = code


class wlc_config(ct.Structure):
    _fields_ = [("n_z", ct.c_int32), ("n_ell", ct.c_int32), ("n_chi", ct.c_int32), ("n_k", ct.c_int32),
                ("n_m", ct.c_int32), ("tomo_mode", ct.c_int32), ("precision", ct.c_int32), ("flags", ct.c_int32),
                ("ell_min", ct.c_double), ("ell_max", ct.c_double), ("ell_cut", ct.c_double),
                ("f_sky", ct.c_double), ("sigma_eps", ct.c_double), ("n_gal_arcmin2", ct.c_double),
                ("sigma_b2", ct.c_double), ("k_max", ct.c_double), ("rho_mean", ct.c_double),
                ("n_sub", ct.c_int32), ("gram_tol", ct.c_double)]


class wlc_tables(ct.Structure):
    _fields_ = [(n, ct.c_void_p) for n in ("chi", "w_chi", "k", "m", "w_m", "W", "P", "u", "n_m", "b1", "b2",
                                           "n_tri")]


class wlc_sizes(ct.Structure):
    _fields_ = [("n_data", ct.c_int64), ("n_distinct", ct.c_int64), ("n_p", ct.c_int64), ("n_tri", ct.c_int64),
                ("n_cfg", ct.c_int64), ("n_ell_used", ct.c_int64), ("k_len", ct.c_int64),
                ("c_elem_bytes", ct.c_size_t), ("ws_run_bytes", ct.c_size_t), ("ws_snr_bytes", ct.c_size_t),
                ("ws_snr_structured_bytes", ct.c_size_t), ("n_avg", ct.c_int64), ("ws_pca_bytes", ct.c_size_t)]


def _hip_runtimes():
    """Paths of the HIP runtime libraries mapped into this process."""
    try:
        with open("/proc/self/maps") as f:
            return {line.split()[-1] for line in f if "libamdhip64" in line and "/" in line}
    except OSError:
        return set()


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libwlcov.so is not built (run paper_1812_07437_amd.build.build())")
    L = ct.CDLL(LIB_PATH)
    # one HIP runtime per process: with two (libwlcov bound to another copy
    # than torch's), device pointers of one are invalid in the other
    rt = _hip_runtimes()
    if len(rt) > 1:
        raise ImportError("libwlcov and torch loaded different HIP runtimes: %s" % sorted(rt))
    vp = ct.c_void_p
    L.wlc_last_error.restype = ct.c_char_p
    L.wlc_plan_create.argtypes = [ct.POINTER(wlc_config), ct.POINTER(vp)]
    L.wlc_plan_destroy.argtypes = [vp]
    L.wlc_plan_destroy.restype = None
    L.wlc_plan_sizes.argtypes = [vp, ct.POINTER(wlc_sizes)]
    L.wlc_plan_index.argtypes = [vp, vp, vp, vp]
    L.wlc_plan_gram_order.argtypes = [vp, vp]
    L.wlc_counts_closed.argtypes = [vp, vp, vp]
    L.wlc_plan_averaging.argtypes = [vp, vp, vp, vp, vp]
    L.wlc_lattice_counts.argtypes = [vp, vp, vp, vp, vp]
    L.wlc_run.argtypes = [vp, ct.POINTER(wlc_tables), vp, vp, vp, vp, vp, vp]
    L.wlc_sigma_w2.argtypes = [vp, ct.POINTER(wlc_tables), vp, vp]
    L.wlc_snr2.argtypes = [vp, vp, vp, vp, vp, ct.POINTER(ct.c_double), vp]
    L.wlc_snr2_structured.argtypes = [vp, vp, vp, ct.POINTER(ct.c_double), vp]
    L.wlc_snr2_lmax.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.wlc_snr2_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.wlc_gram_split_tiles.argtypes = [vp, vp, vp, vp]
    L.wlc_gram_ws_bytes.argtypes = [ct.c_int, ct.c_int64, ct.c_int64, vp]
    L.wlc_gram.argtypes = [ct.c_int, ct.c_int64, ct.c_int64, vp, vp, vp, ct.c_double, vp, vp, vp, vp]
    L.wlc_gram_work.argtypes = [vp, vp, vp, vp, vp]
    L.wlc_pca.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.wlc_plan_set_timing.argtypes = [vp, ct.c_int]
    L.wlc_plan_timings.argtypes = [vp, vp]
    L.wlc_plan_kernel_stats.argtypes = [vp, vp, vp, vp, vp]
    return L


lib = _load()

EXPORTED = ["wlc_plan_create", "wlc_plan_destroy", "wlc_plan_sizes", "wlc_plan_index", "wlc_plan_gram_order",
            "wlc_plan_averaging",
            "wlc_counts_closed",
            "wlc_lattice_counts", "wlc_run", "wlc_sigma_w2", "wlc_snr2", "wlc_snr2_noalloc", "wlc_gram_split_tiles", "wlc_gram_ws_bytes", "wlc_gram", "wlc_gram_work", "wlc_snr2_lmax", "wlc_pca", "wlc_snr2_structured", "wlc_plan_set_timing",
            "wlc_plan_timings",
            "wlc_plan_kernel_stats", "wlc_last_error"]
PHASES = ["tables", "abuild", "gram", "assemble", "snr_prep", "chol"]


def wlc_plan_set_timing(plan, enable):
    _check(lib.wlc_plan_set_timing(plan, int(bool(enable))))


def wlc_plan_timings(plan):
    ms = (ct.c_float * len(PHASES))()
    _check(lib.wlc_plan_timings(plan, ct.cast(ms, ct.c_void_p)))
    return dict(zip(PHASES, [float(x) for x in ms]))


def wlc_plan_kernel_stats(plan):
    ms = ct.c_double(); n = ct.c_int64(); timed = ct.c_int64(); fl = ct.c_double()
    _check(lib.wlc_plan_kernel_stats(plan, ct.byref(ms), ct.byref(n), ct.byref(timed), ct.byref(fl)))
    return dict(ms=ms.value, launches=n.value, timed=timed.value, flops=fl.value)


def wlc_last_error():
    return lib.wlc_last_error().decode()


def _check(rc):
    if rc != WLC_OK:
        raise WlcError(rc, wlc_last_error())


def wlc_plan_create(cfg: wlc_config):
    h = ct.c_void_p()
    _check(lib.wlc_plan_create(ct.byref(cfg), ct.byref(h)))
    return h


def wlc_plan_destroy(plan):
    lib.wlc_plan_destroy(plan)


def wlc_plan_sizes(plan) -> wlc_sizes:
    s = wlc_sizes()
    _check(lib.wlc_plan_sizes(plan, ct.byref(s)))
    return s


def wlc_plan_index(plan, tri, rows, distinct):
    _check(lib.wlc_plan_index(plan, tri, rows, distinct))


def wlc_plan_gram_order(plan, pos):
    _check(lib.wlc_plan_gram_order(plan, pos))


def wlc_plan_averaging(plan, off, legs, ell, w):
    _check(lib.wlc_plan_averaging(plan, off, legs, ell, w))


def wlc_counts_closed(plan, n_modes, n_tri):
    _check(lib.wlc_counts_closed(plan, n_modes, n_tri))


def wlc_lattice_counts(plan, ws, modes, tris, stream):
    _check(lib.wlc_lattice_counts(plan, ws, modes, tris, stream))


def wlc_run(plan, tables: wlc_tables, ws, d, r, C, row_exp2, stream):
    _check(lib.wlc_run(plan, ct.byref(tables), ws, d, r, C, row_exp2, stream))


def wlc_sigma_w2(plan, tables: wlc_tables, sw, stream):
    _check(lib.wlc_sigma_w2(plan, ct.byref(tables), sw, stream))


def wlc_snr2(plan, C, row_exp2, d, ws, stream):
    out = ct.c_double()
    _check(lib.wlc_snr2(plan, C, row_exp2, d, ws, ct.byref(out), stream))
    return out.value


def wlc_snr2_noalloc(plan, C, row_exp2, d, snr2_dev, status_dev, stream):
    """Enqueue (S/N)^2 into DEVICE snr2_dev[0] and the pivot status into DEVICE
    status_dev[0], with the library's fixed scratch (no allocation, no sync)."""
    _check(lib.wlc_snr2_noalloc(plan, C, row_exp2, d, snr2_dev, status_dev, stream))


def wlc_gram_split_tiles(plan, ws_run):
    """(tiles that took the split product, tiles) of the last run."""
    a, b = ct.c_int64(), ct.c_int64()
    _check(lib.wlc_gram_split_tiles(plan, ws_run, ct.byref(a), ct.byref(b)))
    return a.value, b.value


def wlc_gram_ws_bytes(precision, n, k):
    """Workspace bytes of wlc_gram (the split-K partial products)."""
    b = ct.c_size_t()
    _check(lib.wlc_gram_ws_bytes(_prec(precision), int(n), int(k), ct.byref(b)))
    return b.value


def wlc_gram(precision, n, k, a_hi, a_lo, panel_f, lim, g, ws, stream, panel_ext=None):
    """Enqueue the lower 256-tiles of A A^T (FP32, DEVICE g [n_pad][n_pad]) of a
    k-blocked bf16 factor (DEVICE a_hi, a_lo; see include/wlcov.h)."""
    _check(lib.wlc_gram(_prec(precision), int(n), int(k), a_hi, a_lo, panel_f, float(lim), panel_ext, g, ws, stream))


def wlc_gram_work(plan, ws_run):
    """(flops, MFMA flops, factor bytes) of the last run's one-halo product."""
    a, b, c = ct.c_double(), ct.c_double(), ct.c_double()
    _check(lib.wlc_gram_work(plan, ws_run, ct.byref(a), ct.byref(b), ct.byref(c)))
    return a.value, b.value, c.value


def wlc_snr2_lmax(plan, C, row_exp2, d, ws, stream, n_ell):
    import numpy as np
    out = np.zeros(int(n_ell), np.float64)
    _check(lib.wlc_snr2_lmax(plan, C, row_exp2, d, ws, out.ctypes.data_as(ct.c_void_p), stream))
    return out


def wlc_pca(plan, C, row_exp2, d, ws, n, S, stream):
    """Returns (lambda, snr2_mode, cum_desc, sweeps) as numpy arrays / int."""
    import numpy as np
    lam = np.zeros(int(n)); snr = np.zeros(int(n)); cum = np.zeros(int(n)); sw = ct.c_int32(0)
    _check(lib.wlc_pca(plan, C, row_exp2, d, ws, lam.ctypes.data_as(ct.c_void_p), snr.ctypes.data_as(ct.c_void_p),
                       cum.ctypes.data_as(ct.c_void_p), ct.byref(sw), S, stream))
    return lam, snr, cum, sw.value


def wlc_snr2_structured(plan, ws_run, ws, stream):
    out = ct.c_double()
    _check(lib.wlc_snr2_structured(plan, ws_run, ws, ct.byref(out), stream))
    return out.value


# ---------------------------------------------------------------- helpers
def make_config(cfg: dict, precision="fp64", tomo="paper", nocheck=False, ngins=False,
                ssc_chi=False, n_sub=0, gram_tol=0.0) -> wlc_config:
    """wlc_config from a dict of scalars (n_z, n_ell, n_chi, n_k, n_m, ell_min,
    ell_max, f_sky, sigma_eps, n_gal_arcmin2, sigma_b2, k_max, rho_mean and
    optionally ell_cut); ngins adds the B.B, P.T and P.B terms, ssc_chi
    resolves the super-sample term along the line of sight, n_sub > 1
    averages every polyspectrum over n_sub sub-bins per ell-bin."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    flags = (WLC_FLAG_NOCHECK if nocheck else 0) | (WLC_FLAG_NGINS if ngins else 0) | \
        (WLC_FLAG_SSC_CHI if ssc_chi else 0)
    return wlc_config(n_z=int(cfg["n_z"]), n_ell=int(cfg["n_ell"]), n_chi=int(cfg["n_chi"]), n_k=int(cfg["n_k"]),
                      n_m=int(cfg["n_m"]), tomo_mode=WLC_TOMO_SORTED if tomo == "sorted" else WLC_TOMO_PAPER,
                      precision=prec, flags=flags,
                      ell_min=float(cfg["ell_min"]), ell_max=float(cfg["ell_max"]),
                      ell_cut=float(cfg.get("ell_cut", 0.0) or 0.0), f_sky=float(cfg["f_sky"]),
                      sigma_eps=float(cfg["sigma_eps"]), n_gal_arcmin2=float(cfg["n_gal_arcmin2"]),
                      sigma_b2=float(cfg["sigma_b2"]), k_max=float(cfg["k_max"]), rho_mean=float(cfg["rho_mean"]),
                      n_sub=int(n_sub), gram_tol=float(gram_tol))


def _ptr(t):
    return ct.c_void_p(t.data_ptr()) if t is not None else None


def _stream_handle(stream):
    return ct.c_void_p(stream.cuda_stream) if stream is not None else None


class Problem:
    """One plan plus device-resident tables, workspace and outputs.

    ``arrays`` maps the table names of wlc_tables (chi, w_chi, k, m, w_m, W, P,
    u, n_m, optional b1, b2, n_tri) to float64 arrays (numpy or torch)."""

    def __init__(self, cfg: dict, arrays: dict, precision="fp64", tomo="paper", device="cuda:0",
                 nocheck=False, ngins=False, ssc_chi=False, n_sub=0, gram_tol=0.0):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.config = make_config(cfg, precision, tomo, nocheck, ngins, ssc_chi, n_sub, gram_tol)
        self.plan = wlc_plan_create(self.config)
        self.sizes = wlc_plan_sizes(self.plan)
        self._tabs = {}
        for name in ("chi", "w_chi", "k", "m", "w_m", "W", "P", "u", "n_m", "b1", "b2", "n_tri"):
            a = arrays.get(name)
            if a is None:
                self._tabs[name] = None
                continue
            t = torch.as_tensor(a, dtype=torch.float64).contiguous().to(self.device)
            self._tabs[name] = t
        self.tables = wlc_tables(**{k: (_ptr(v) if v is not None else None) for k, v in self._tabs.items()})
        n = self.sizes.n_data
        cdt = torch.float64 if self.sizes.c_elem_bytes == 8 else torch.float32
        self.d = torch.empty(n, dtype=torch.float64, device=self.device)
        self.r = torch.empty(n, dtype=torch.float64, device=self.device)
        self.C = torch.empty((n, n), dtype=cdt, device=self.device)
        self.row_exp2 = torch.empty(n, dtype=torch.int32, device=self.device)
        self.ws = torch.empty(int(self.sizes.ws_run_bytes), dtype=torch.uint8, device=self.device)
        self.ws_snr = None

    def close(self):
        if self.plan:
            wlc_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, stream=None):
        wlc_run(self.plan, self.tables, _ptr(self.ws), _ptr(self.d), _ptr(self.r), _ptr(self.C),
                _ptr(self.row_exp2), _stream_handle(stream))

    def sigma_w2(self, stream=None):
        """sigma_W^2 at every chi node of this problem's tables (device)."""
        sw = self.torch.empty(int(self.config.n_chi), dtype=self.torch.float64, device=self.device)
        wlc_sigma_w2(self.plan, self.tables, _ptr(sw), _stream_handle(stream))
        return sw

    def snr2(self, stream=None):
        if self.ws_snr is None:
            self.ws_snr = self.torch.empty(int(self.sizes.ws_snr_bytes), dtype=self.torch.uint8, device=self.device)
        return wlc_snr2(self.plan, _ptr(self.C), _ptr(self.row_exp2), _ptr(self.d), _ptr(self.ws_snr),
                        _stream_handle(stream))

    def snr2_noalloc(self, out, status, stream=None):
        """Enqueue (S/N)^2 into the device tensors out (float64) and status
        (int32), one element each, through the fixed-scratch entry point."""
        wlc_snr2_noalloc(self.plan, _ptr(self.C), _ptr(self.row_exp2), _ptr(self.d), _ptr(out), _ptr(status),
                         _stream_handle(stream))

    def split_tiles(self):
        """(split, total) tiles of this problem's last run's one-halo product."""
        self.torch.cuda.synchronize()
        return wlc_gram_split_tiles(self.plan, _ptr(self.ws))

    def gram_work(self):
        """(flops, MFMA flops, factor bytes) of the last run's one-halo product."""
        return wlc_gram_work(self.plan, _ptr(self.ws))

    def snr2_lmax(self, stream=None):
        """(S/N)^2 of the data vector cut after each ell-bin (numpy array)."""
        if self.ws_snr is None:
            self.ws_snr = self.torch.empty(int(self.sizes.ws_snr_bytes), dtype=self.torch.uint8, device=self.device)
        return wlc_snr2_lmax(self.plan, _ptr(self.C), _ptr(self.row_exp2), _ptr(self.d), _ptr(self.ws_snr),
                             _stream_handle(stream), self.sizes.n_ell_used)

    def pca(self, vectors=True, stream=None):
        """Principal components of this problem's covariance: (lambda,
        snr2_mode, cum_desc, sweeps, S or None), S a device tensor."""
        n = int(self.sizes.ws_pca_bytes)
        if n == 0:
            raise WlcError(WLC_EINVAL, "PCA not available for this plan size")
        ws = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
        N = int(self.sizes.n_data)
        S = self.torch.empty((N, N), dtype=self.torch.float64, device=self.device) if vectors else None
        lam, snr, cum, sw = wlc_pca(self.plan, _ptr(self.C), _ptr(self.row_exp2), _ptr(self.d), _ptr(ws), N,
                                    _ptr(S), _stream_handle(stream))
        del ws
        return lam, snr, cum, sw, S

    def snr2_structured(self, stream=None):
        """(S/N)^2 through the distinct rows, from this problem's last run."""
        if getattr(self, "ws_struct", None) is None:
            n = int(self.sizes.ws_snr_structured_bytes)
            if n == 0:
                raise WlcError(WLC_EINVAL, "structured S/N not available for this plan")
            self.ws_struct = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
        return wlc_snr2_structured(self.plan, _ptr(self.ws), _ptr(self.ws_struct), _stream_handle(stream))

    def free_snr_workspace(self):
        self.ws_snr = None
        self.ws_struct = None

    def covariance_true(self):
        """C_true = C * 2^-(t_a + t_b) in float64 (host numpy)."""
        import numpy as np
        C = self.C.double().cpu().numpy()
        t = self.row_exp2.cpu().numpy().astype(np.int64)
        return np.ldexp(C, -(t[:, None] + t[None, :]))

    def index(self):
        import numpy as np
        s = self.sizes
        tri = np.zeros((max(1, s.n_tri), 3), np.int32)
        rows = np.zeros((s.n_data, 8), np.int32)
        distinct = np.zeros(s.n_data, np.int32)
        wlc_plan_index(self.plan, tri.ctypes.data_as(ct.c_void_p), rows.ctypes.data_as(ct.c_void_p),
                       distinct.ctypes.data_as(ct.c_void_p))
        return tri[:s.n_tri], rows, distinct

    def gram_order(self):
        """pos[e]: the row of the one-halo product that holds distinct row e."""
        import numpy as np
        pos = np.zeros(self.sizes.n_distinct, np.int32)
        wlc_plan_gram_order(self.plan, pos.ctypes.data_as(ct.c_void_p))
        return pos

    def lattice_counts(self, stream=None):
        torch = self.torch
        modes = torch.zeros(self.sizes.n_ell_used, dtype=torch.int64, device=self.device)
        tris = torch.zeros(max(1, self.sizes.n_tri), dtype=torch.int64, device=self.device)
        wlc_lattice_counts(self.plan, _ptr(self.ws), _ptr(modes), _ptr(tris), _stream_handle(stream))
        return modes, tris[:self.sizes.n_tri]
