"""ctypes binding of the libwlcov request server (include/wlcov_serve.h).

Argument marshalling only; the scheduling, admission and every kernel run in
the library.  Tables and result buffers are torch tensors on the device.
"""
from __future__ import annotations

import ctypes as ct

from .wlcov import PRECISIONS, WlcError, _check, _ptr, _stream_handle, lib, make_config, wlc_tables


class wlc_request(ct.Structure):
    _fields_ = [("n_z", ct.c_int32), ("precision", ct.c_int32), ("snr_method", ct.c_int32), ("pad", ct.c_int32),
                ("ell_max", ct.c_double),
                ("p_scale", ct.c_double), ("n_scale", ct.c_double), ("rho_mean", ct.c_double),
                ("W", ct.c_void_p)]


class wlc_result(ct.Structure):
    _fields_ = [("status", ct.c_int32), ("pad", ct.c_int32), ("n_data", ct.c_int64), ("c_elem_bytes", ct.c_size_t),
                ("snr2", ct.c_double), ("t_submit_ms", ct.c_double), ("t_admit_ms", ct.c_double),
                ("t_done_ms", ct.c_double), ("d", ct.c_void_p), ("r", ct.c_void_p), ("C", ct.c_void_p),
                ("row_exp2", ct.c_void_p)]


class wlc_server_stats(ct.Structure):
    _fields_ = [("queued", ct.c_int64), ("running", ct.c_int64), ("done", ct.c_int64),
                ("arena_bytes", ct.c_size_t), ("arena_used", ct.c_size_t), ("arena_peak", ct.c_size_t),
                ("completed_total", ct.c_int64), ("batches", ct.c_int64), ("batched_requests", ct.c_int64),
                ("max_batch", ct.c_int64)]


SNR_METHODS = {"direct": 0, "structured": 1}

vp = ct.c_void_p
lib.wlc_server_create.argtypes = [vp, vp, ct.c_size_t, ct.c_int32, ct.POINTER(vp)]
lib.wlc_server_submit.argtypes = [vp, ct.POINTER(wlc_request), ct.POINTER(ct.c_uint64)]
lib.wlc_server_poll.argtypes = [vp, ct.c_uint64, ct.POINTER(ct.c_int32), ct.POINTER(wlc_result)]
lib.wlc_server_wait.argtypes = [vp, ct.c_uint64, ct.POINTER(wlc_result)]
lib.wlc_server_copy.argtypes = [vp, ct.c_uint64, vp, vp, vp, vp, vp]
lib.wlc_server_release.argtypes = [vp, ct.c_uint64]
lib.wlc_server_get_stats.argtypes = [vp, ct.POINTER(wlc_server_stats)]
lib.wlc_server_destroy.argtypes = [vp]

EXPORTED = ["wlc_server_create", "wlc_server_submit", "wlc_server_poll", "wlc_server_wait", "wlc_server_copy",
            "wlc_server_release", "wlc_server_get_stats", "wlc_server_destroy"]


def wlc_server_create(cfg, tables, hbm_budget, max_inflight):
    h = ct.c_void_p()
    _check(lib.wlc_server_create(ct.byref(cfg), ct.byref(tables), int(hbm_budget), int(max_inflight), ct.byref(h)))
    return h


def wlc_server_submit(srv, req):
    t = ct.c_uint64()
    _check(lib.wlc_server_submit(srv, ct.byref(req), ct.byref(t)))
    return t.value


def wlc_server_poll(srv, ticket):
    done = ct.c_int32()
    res = wlc_result()
    _check(lib.wlc_server_poll(srv, ticket, ct.byref(done), ct.byref(res)))
    return bool(done.value), res


def wlc_server_wait(srv, ticket):
    res = wlc_result()
    _check(lib.wlc_server_wait(srv, ticket, ct.byref(res)))
    return res


def wlc_server_copy(srv, ticket, d, r, C, row_exp2, stream):
    _check(lib.wlc_server_copy(srv, ticket, d, r, C, row_exp2, stream))


def wlc_server_release(srv, ticket):
    _check(lib.wlc_server_release(srv, ticket))


def wlc_server_get_stats(srv):
    s = wlc_server_stats()
    _check(lib.wlc_server_get_stats(srv, ct.byref(s)))
    return s


def wlc_server_destroy(srv):
    _check(lib.wlc_server_destroy(srv))


class Server:
    """Owns the device-resident fiducial tables and a server handle."""

    def __init__(self, cfg: dict, arrays: dict, hbm_budget: int, max_inflight=4, precision="bf16x3",
                 device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.cfg = dict(cfg)
        self.n_chi = int(cfg["n_chi"])
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        base = make_config(cfg, precision)
        self._tabs = {}
        for name in ("chi", "w_chi", "k", "m", "w_m", "P", "u", "n_m", "b1", "b2", "n_tri"):
            a = arrays.get(name)
            self._tabs[name] = None if a is None else torch.as_tensor(a, dtype=torch.float64).contiguous().to(
                self.device)
        ptrs = {k: (_ptr(v) if v is not None else None) for k, v in self._tabs.items()}
        ptrs["W"] = None
        self.tables = wlc_tables(**ptrs)
        self.handle = wlc_server_create(base, self.tables, hbm_budget, max_inflight)

    def submit(self, W, n_z, ell_max, p_scale=1.0, n_scale=1.0, rho_mean=None, precision=None, snr="direct"):
        """snr: "direct" (Cholesky of the whole covariance) or "structured"
        (through the distinct rows)."""
        import numpy as np
        W = np.ascontiguousarray(W, dtype=np.float64)
        assert W.shape == (n_z, self.n_chi)
        req = wlc_request(n_z=int(n_z), precision=self.precision if precision is None else
                          (PRECISIONS[precision] if isinstance(precision, str) else int(precision)),
                          snr_method=SNR_METHODS[snr] if isinstance(snr, str) else int(snr),
                          ell_max=float(ell_max), p_scale=float(p_scale), n_scale=float(n_scale),
                          rho_mean=float(rho_mean if rho_mean is not None else self.cfg["rho_mean"]),
                          W=W.ctypes.data_as(ct.c_void_p))
        return wlc_server_submit(self.handle, req)

    def poll(self, ticket):
        return wlc_server_poll(self.handle, ticket)

    def wait(self, ticket):
        return wlc_server_wait(self.handle, ticket)

    def fetch(self, ticket):
        """Copies of a finished request's (d, r, C, row_exp2) as device tensors."""
        torch = self.torch
        res = self.wait(ticket)
        n = res.n_data
        d = torch.empty(n, dtype=torch.float64, device=self.device)
        r = torch.empty(n, dtype=torch.float64, device=self.device)
        C = torch.empty((n, n), dtype=torch.float64 if res.c_elem_bytes == 8 else torch.float32, device=self.device)
        t = torch.empty(n, dtype=torch.int32, device=self.device)
        stream = torch.cuda.current_stream()
        wlc_server_copy(self.handle, ticket, _ptr(d), _ptr(r), _ptr(C), _ptr(t), _stream_handle(stream))
        torch.cuda.synchronize()
        return res, d, r, C, t

    def release(self, ticket):
        wlc_server_release(self.handle, ticket)

    def stats(self):
        return wlc_server_get_stats(self.handle)

    def close(self):
        if self.handle:
            wlc_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
