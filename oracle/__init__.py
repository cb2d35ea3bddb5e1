"""FP64 CPU oracle for the weak-lensing P+B data vector, covariance and S/N.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; nothing in the product package
imports it.  It shares no code with the HIP library.

The combinatorics (ell-bins, triangles, tomographic orderings, counts) are
plain Python here; the heavy sums are plain C in ``wlc_oracle.c`` (built with
gcc, loaded through ctypes).  Each function cites the passage of Rizzato et
al. (2019), arXiv 1812.07437, that it writes out.

Parity unpinned: the B_G2 term of the bispectrum response (eq. RespB).  The
paper never defines B_G2; the tidal-kernel reading in ``wlc_oracle.c`` is
checked only against its own closed-form values, not against the paper.
"""
from __future__ import annotations

import ctypes as ct
import math
import os
import subprocess
from itertools import product

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wlc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force=False):
    """Compile the C part of the oracle (gcc -O3 -fopenmp)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class _Tables(ct.Structure):
    _fields_ = [("n_z", ct.c_int), ("n_chi", ct.c_int), ("n_k", ct.c_int), ("n_m", ct.c_int),
                ("chi", ct.c_void_p), ("w_chi", ct.c_void_p), ("k", ct.c_void_p),
                ("m", ct.c_void_p), ("w_m", ct.c_void_p), ("W", ct.c_void_p), ("P", ct.c_void_p),
                ("u", ct.c_void_p), ("nmf", ct.c_void_p), ("b1", ct.c_void_p), ("b2", ct.c_void_p),
                ("rho", ct.c_double), ("k_max", ct.c_double)]


def lib():
    global _lib
    if _lib is None:
        build()
        L = ct.CDLL(_LIB)
        L.or_interp.restype = ct.c_double
        L.or_neff.restype = ct.c_double
        L.or_halo_I.restype = ct.c_double
        L.or_F2.restype = ct.c_double
        L.or_lattice_modes.restype = ct.c_uint64
        L.or_lattice_triangles.restype = ct.c_uint64
        L.or_lattice_modes.argtypes = [ct.c_int64] * 2
        L.or_lattice_triangles.argtypes = [ct.c_int64] * 6
        L.or_F2.argtypes = [ct.c_double] * 3
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ct.c_void_p) if a is not None else None


# ===================================================================
# Combinatorics (Sec. 3.2.1, Sec. 5, App. A)
# ===================================================================
def ell_bins(ell_min, ell_max, n_ell):
    """Bins equally spaced in log ell (Sec. 3.2.1, App. A).  Each bin is the
    symmetric interval of width Delta around its centre, so the centre is the
    arithmetic mid-point of its two edges."""
    a, b = math.log(ell_min), math.log(ell_max)
    edges = [math.exp(a + i * (b - a) / n_ell) for i in range(n_ell + 1)]
    centres = [(edges[i] + edges[i + 1]) / 2.0 for i in range(n_ell)]
    widths = [edges[i + 1] - edges[i] for i in range(n_ell)]
    return edges, centres, widths


def n_ell_used(centres, ell_cut):
    """Bins kept when the S/N is cut at ell_max (eq. eq:SN): those whose
    centre lies below the cut; all bins when there is no cut."""
    if not ell_cut or ell_cut <= 0:
        return len(centres)
    return sum(1 for c in centres if c < ell_cut)


def triangles(centres):
    """Binned triangles l_i <= l_j <= l_k in data-vector order (Sec. 5: j runs
    fastest, k slowest; i in between).  A bin triplet is a triangle when its
    centres obey the strict triangle inequality.  Returns (i, j, k, class)
    with class 'E' (all equal), 'I' (two equal) or 'S' (all different)."""
    out = []
    n = len(centres)
    for k in range(n):
        for i in range(k + 1):
            for j in range(i, k + 1):
                if centres[i] + centres[j] > centres[k]:
                    cls = "E" if i == j == k else ("I" if (i == j or j == k) else "S")
                    out.append((i, j, k, cls))
    return out


def bispectrum_tomo(n_z, tri):
    """Tomographic bin triplets of one triangle, k fastest and i slowest
    (Sec. 5).  Scalene triangles keep all n_z^3 combinations; when two sides
    share an ell-bin only one ordering of their redshift bins is kept, since
    swapping those two legs leaves the bispectrum unchanged."""
    i, j, k, cls = tri
    out = []
    for a, b, c in product(range(n_z), repeat=3):
        if cls == "S":
            out.append((a, b, c))
        elif cls == "E":
            if a <= b <= c:
                out.append((a, b, c))
        elif i == j:          # l1 = l2 < l3
            if a <= b:
                out.append((a, b, c))
        else:                 # l1 < l2 = l3
            if b <= c:
                out.append((a, b, c))
    return out


def enumerate_rows(n_z, n_ell, centres, tomo="paper"):
    """Data vector D = {P, B} (eq. eq:SN2, Sec. 5).  P block: ell-bins in
    increasing order, pairs i <= j with j fastest.  B block: triangles in the
    order above, each with its tomographic triplets contiguous.  With
    tomo="sorted" every triangle keeps only triplets i <= j <= k.

    Returns dict of numpy arrays kind, lbin[N,3], zbin[N,3], cfg, tri and the
    triangle list.  cfg indexes the ell-configuration: the ell-bin for P rows,
    n_ell + triangle index for B rows."""
    cen = centres[:n_ell]
    tris = triangles(cen)
    kind, lbin, zbin, cfg, tri = [], [], [], [], []
    for b in range(n_ell):
        for i in range(n_z):
            for j in range(i, n_z):
                kind.append(2); lbin.append((b, b, -1)); zbin.append((i, j, -1))
                cfg.append(b); tri.append(-1)
    for t, trg in enumerate(tris):
        trip = bispectrum_tomo(n_z, trg) if tomo == "paper" else \
            [(a, b, c) for a in range(n_z) for b in range(a, n_z) for c in range(b, n_z)]
        for (a, b, c) in trip:
            kind.append(3); lbin.append(trg[:3]); zbin.append((a, b, c))
            cfg.append(n_ell + t); tri.append(t)
    return dict(kind=np.array(kind, np.int32), lbin=np.array(lbin, np.int32),
                zbin=np.array(zbin, np.int32), cfg=np.array(cfg, np.int32),
                tri=np.array(tri, np.int32), triangles=tris)


def canonical_rows(rows):
    """Row value classes.  Under Limber every bin sees the same chi, so a
    row's data-vector value, response and one-halo covariance depend only on
    its ell-configuration and the multiset of its redshift bins.  Returns
    (canon[N] -> class id, index of one representative row per class)."""
    key_to_id, canon, reps = {}, [], []
    for a in range(len(rows["kind"])):
        p = int(rows["kind"][a])
        key = (int(rows["cfg"][a]), tuple(sorted(int(x) for x in rows["zbin"][a][:p])))
        if key not in key_to_id:
            key_to_id[key] = len(reps)
            reps.append(a)
        canon.append(key_to_id[key])
    return np.array(canon, np.int32), np.array(reps, np.int64)


# ===================================================================
# Counts (Sec. 3.2.2, App. B)
# ===================================================================
def n_modes(centres, widths, f_sky):
    """N(l_b) = 2 l Delta l f_sky (Sec. 3.2.2), read as a number of modes."""
    return [2.0 * c * w * f_sky for c, w in zip(centres, widths)]


def n_tri_closed(l1, l2, l3, d1, d2, d3, f_sky):
    """Continuum triangle count at the bin centres (App. B).  The printed
    closed form is garbled; this is the count its own definition gives with a
    mode density Omega/(2 pi)^2:
        N_tri = Omega^2 l1 l2 l3 D1 D2 D3 / (2 pi^3 Lambda),
        Lambda = sqrt(2 l1^2 l2^2 + 2 l1^2 l3^2 + 2 l2^2 l3^2 - l1^4 - l2^4 - l3^4)."""
    om = 4.0 * math.pi * f_sky
    lam2 = 2 * l1 ** 2 * l2 ** 2 + 2 * l1 ** 2 * l3 ** 2 + 2 * l2 ** 2 * l3 ** 2 - l1 ** 4 - l2 ** 4 - l3 ** 4
    if lam2 <= 0:
        raise ValueError("degenerate triangle")
    return om ** 2 * l1 * l2 * l3 * d1 * d2 * d3 / (2.0 * math.pi ** 3 * math.sqrt(lam2))


def sub_bin_centres(edges, centres, n_ell, S):
    """Centres of S equal-width sub-bins of each of the first n_ell ell-bins,
    bin b owning entries b S .. b S + S - 1 (the bin centres when S = 1)."""
    if S == 1:
        return list(centres[:n_ell])
    out = []
    for b in range(n_ell):
        w = edges[b + 1] - edges[b]
        out.extend(edges[b] + (s + 0.5) * w / S for s in range(S))
    return out


def cell_pairs(a1, b1, a2, b2, a3, b3, n=8):
    """Continuum number of ordered mode pairs (l1, l2) with |l1| in [a1, b1),
    |l2| in [a2, b2) and |l1 + l2| in [a3, b3), up to the constant
    (Omega / (2 pi)^2)^2 2 pi: the triangle count of App. B (a sum of the
    selection function) in the continuum.  With phi the angle between the
    modes, |l1 + l2|^2 = l1^2 + l2^2 + 2 l1 l2 cos phi, so the angles in the
    cell form an interval of cos phi, integrated exactly; l1 and l2 by
    Gauss-Legendre on n x n nodes."""
    x, w = np.polynomial.legendre.leggauss(n)
    total = 0.0
    for xi, wi in zip(x, w):
        l1 = 0.5 * (a1 + b1) + 0.5 * (b1 - a1) * xi
        for xj, wj in zip(x, w):
            l2 = 0.5 * (a2 + b2) + 0.5 * (b2 - a2) * xj
            lo = min(1.0, max(-1.0, (a3 * a3 - l1 * l1 - l2 * l2) / (2 * l1 * l2)))
            hi = min(1.0, max(-1.0, (b3 * b3 - l1 * l1 - l2 * l2) / (2 * l1 * l2)))
            dphi = 2.0 * (math.acos(lo) - math.acos(hi))
            total += 0.25 * (b1 - a1) * (b2 - a2) * wi * wj * l1 * l2 * dphi
    return total


def averaging_lists(kinds, legs, S, sub_c, widths):
    """The binned estimators average over the modes of each bin (Sec. 3.2.2)
    and over the triangles of each triangle bin (App. B); the paper takes
    the bin centres instead.  With S sub-bins per side: a power-spectrum bin
    averages over its sub-bins weighted by their number of modes (2 l dl
    f_sky, so proportional to l at equal widths); a triangle bin over the
    cells of sub-bin triples whose centres obey the strict triangle
    inequality, weighted by the continuum count of mode pairs in the cell
    (cell_pairs), with the polyspectra taken at the cell centres.  Returns,
    per configuration, (legs [E][3] as sub-bin indices, weights [E] summing
    to one); S = 1 gives the bin centres with weight 1."""
    out = []
    for kind, lg in zip(kinds, legs):
        if S == 1:
            L = [(lg[0], lg[0], lg[0]) if kind == 2 else tuple(lg)]
            W = [1.0]
        elif kind == 2:
            L = [(lg[0] * S + s,) * 3 for s in range(S)]
            W = [sub_c[lg[0] * S + s] for s in range(S)]
        else:
            L, W = [], []
            for s1 in range(S):
                for s2 in range(S):
                    for s3 in range(S):
                        g = (lg[0] * S + s1, lg[1] * S + s2, lg[2] * S + s3)
                        l1, l2, l3 = (sub_c[x] for x in g)
                        if not (l1 < l2 + l3 and l2 < l1 + l3 and l3 < l1 + l2):
                            continue
                        h = [widths[lg[q]] / S / 2 for q in range(3)]
                        n = cell_pairs(l1 - h[0], l1 + h[0], l2 - h[1], l2 + h[1], l3 - h[2], l3 + h[2])
                        if n > 0:
                            L.append(g)
                            W.append(n)
            if not L:
                raise ValueError("a binned triangle has no sub-bin triangle")
        W = np.array(W, np.float64)
        out.append((np.array(L, np.int32), W / W.sum() if S > 1 else W))
    return out


def lattice_thresholds(edges, f_sky):
    """Integer thresholds on |q|^2 for the mode lattice: fundamental mode
    l_f = 2 pi / sqrt(Omega) (a square patch of area Omega; reading of
    Sec. 3.2.2), bin b holds q with ceil((e_b/l_f)^2) <= |q|^2 < ceil((e_{b+1}/l_f)^2)."""
    om = 4.0 * math.pi * f_sky
    lf = 2.0 * math.pi / math.sqrt(om)
    return [int(math.ceil((e / lf) ** 2)) for e in edges]


def lattice_modes(thr, b):
    return int(lib().or_lattice_modes(thr[b], thr[b + 1]))


def lattice_triangles(thr, b1, b2, b3):
    """Ordered pairs (q1, q2) with q1 in b1, q2 in b2, q1 + q2 in b3 (App. B,
    definition of N_tri as the sum of the selection function)."""
    return int(lib().or_lattice_triangles(thr[b1], thr[b1 + 1], thr[b2], thr[b2 + 1],
                                          thr[b3], thr[b3 + 1]))


# ===================================================================
# Numerics (C)
# ===================================================================
class Oracle:
    """Holds one set of input tables and evaluates the method on them."""

    def __init__(self, tables, tomo="paper", n_sub=1):
        self.t = tables
        cfg = tables.cfg
        self.cfg = cfg
        self.n_z = int(cfg["n_z"])
        edges, centres, widths = ell_bins(cfg["ell_min"], cfg["ell_max"], int(cfg["n_ell"]))
        self.n_ell = n_ell_used(centres, cfg.get("ell_cut", 0.0))
        self.edges, self.centres, self.widths = edges, centres, widths
        self.rows = enumerate_rows(self.n_z, self.n_ell, centres, tomo)
        self.tris = self.rows["triangles"]
        self.N = len(self.rows["kind"])
        self.f_sky = float(cfg["f_sky"])
        self.omega = 4.0 * math.pi * self.f_sky
        self._keep = []
        arr = {}
        for name in ("chi", "w_chi", "k", "m", "w_m", "W", "P", "u", "n_m", "b1", "b2"):
            a = getattr(tables, name)
            if a is not None:
                a = np.ascontiguousarray(a, dtype=np.float64)
                self._keep.append(a)
            arr[name] = a
        self.arr = arr
        self.T = _Tables(n_z=self.n_z, n_chi=len(arr["chi"]), n_k=len(arr["k"]), n_m=len(arr["m"]),
                         chi=_p(arr["chi"]), w_chi=_p(arr["w_chi"]), k=_p(arr["k"]), m=_p(arr["m"]),
                         w_m=_p(arr["w_m"]), W=_p(arr["W"]), P=_p(arr["P"]), u=_p(arr["u"]),
                         nmf=_p(arr["n_m"]), b1=_p(arr["b1"]), b2=_p(arr["b2"]),
                         rho=float(cfg["rho_mean"]), k_max=float(cfg["k_max"]))
        self.n_chi = len(arr["chi"])
        self.n_m = len(arr["m"])
        self._spectra = None
        self._U = None
        # bin averaging over n_sub sub-bins per side (1: bin centres)
        self.n_sub = max(1, int(n_sub))
        self.sub_c = sub_bin_centres(edges, centres, self.n_ell, self.n_sub)
        kinds, _ = self.configs()
        cl = [(b, b, -1) for b in range(self.n_ell)] + [t[:3] for t in self.tris]
        self.avg = averaging_lists(kinds, cl, self.n_sub, self.sub_c, widths)
        self._Usub = None

    # ---- ell-configurations
    def configs(self):
        kinds, ells = [], []
        for b in range(self.n_ell):
            kinds.append(2); ells.append((self.centres[b], 0.0, 0.0))
        for (i, j, k, _) in self.tris:
            kinds.append(3); ells.append((self.centres[i], self.centres[j], self.centres[k]))
        return np.array(kinds, np.int32), np.array(ells, np.float64)

    def _check(self):
        if lib().or_range_error():
            lib().or_clear_error()
            raise ValueError("a needed k = ell/chi lies outside the k table")

    def spectra(self):
        """3-D spectra and responses at every (configuration, chi) node (bin
        averages when n_sub > 1)."""
        if self._spectra is None and self.n_sub > 1:
            self._spectra = self.spectra_avg()
        if self._spectra is None:
            kinds, ells = self.configs()
            nc = len(kinds)
            X = np.zeros((nc, self.n_chi)); R = np.zeros((nc, self.n_chi))
            lib().or_clear_error()
            lib().or_spectra_table(ct.byref(self.T), ct.c_int(nc), _p(kinds), _p(ells), _p(X), _p(R))
            self._check()
            self._spectra = (X, R)
        return self._spectra

    def spectra_avg(self):
        """X and R averaged over each configuration's averaging list: every
        entry's ell-triple evaluated like a configuration of its own, then
        the weighted sum."""
        kinds, _ = self.configs()
        ke, le, owner, we = [], [], [], []
        for c, (L, W) in enumerate(self.avg):
            for g, w in zip(L, W):
                ke.append(kinds[c])
                le.append((self.sub_c[g[0]], self.sub_c[g[1]], self.sub_c[g[2]]) if kinds[c] == 3
                          else (self.sub_c[g[0]], 0.0, 0.0))
                owner.append(c)
                we.append(w)
        ke = np.array(ke, np.int32)
        le = np.array(le, np.float64)
        Xe = np.zeros((len(ke), self.n_chi)); Re = np.zeros((len(ke), self.n_chi))
        lib().or_clear_error()
        lib().or_spectra_table(ct.byref(self.T), ct.c_int(len(ke)), _p(ke), _p(le), _p(Xe), _p(Re))
        self._check()
        X = np.zeros((len(kinds), self.n_chi)); R = np.zeros((len(kinds), self.n_chi))
        for e, c in enumerate(owner):
            X[c] += we[e] * Xe[e]
            R[c] += we[e] * Re[e]
        return X, R

    def u_table_sub(self):
        """u(m, l_s / chi_n) at every sub-bin centre."""
        if self._Usub is None:
            ell = np.array(self.sub_c, np.float64)
            U = np.zeros((len(ell), self.n_chi, self.n_m))
            lib().or_clear_error()
            lib().or_tab_u(ct.byref(self.T), ct.c_int(len(ell)), _p(ell), _p(U))
            self._check()
            self._Usub = (ell, U)
        return self._Usub

    def cov1h_avg_pairs(self, pairs):
        """One-halo covariance averaged over both rows' averaging lists."""
        ell, U = self.u_table_sub()
        off = np.zeros(len(self.avg) + 1, np.int32)
        for c, (L, _) in enumerate(self.avg):
            off[c + 1] = off[c] + len(L)
        leg = np.ascontiguousarray(np.concatenate([L for L, _ in self.avg]), np.int32)
        w = np.ascontiguousarray(np.concatenate([W for _, W in self.avg]), np.float64)
        pairs = np.ascontiguousarray(pairs, np.int64)
        out = np.zeros(len(pairs))
        lib().or_cov1h_avg_pairs(ct.byref(self.T), _p(ell), _p(U), ct.c_double(self.omega),
                                 _p(np.ascontiguousarray(self.rows["kind"], np.int32)),
                                 _p(np.ascontiguousarray(self.rows["zbin"], np.int32)),
                                 _p(np.ascontiguousarray(self.rows["cfg"], np.int32)), _p(off), _p(leg), _p(w),
                                 ct.c_int64(len(pairs)), _p(pairs), _p(out))
        return out

    def data_vector(self, rows=None):
        """(D, r): eq. nProjection of the halo-model spectra (data vector) and
        of their responses (the projected response of eq. WLSSCflatskyLimber)."""
        rows = rows or self.rows
        X, R = self.spectra()
        n = len(rows["kind"])
        d = np.zeros(n); r = np.zeros(n)
        zb = np.ascontiguousarray(rows["zbin"], np.int32)
        lib().or_project(ct.byref(self.T), ct.c_int(n), _p(rows["kind"]), _p(zb), _p(rows["cfg"]),
                         _p(X), _p(R), _p(d), _p(r))
        return d, r

    def shot_noise(self):
        """sigma_eps^2 / n_i (eq. ShotNoise); equipopulated bins hold n_tot/n_z
        sources per steradian each."""
        nbar = float(self.cfg["n_gal_arcmin2"]) * (10800.0 / math.pi) ** 2 / self.n_z
        return float(self.cfg["sigma_eps"]) ** 2 / nbar

    def ps_table(self):
        """P^s_ij(l_b) for all bins and pairs (eq. ShotNoise)."""
        d, _ = self.data_vector()
        ps = np.zeros((self.n_ell, self.n_z, self.n_z))
        a = 0
        for b in range(self.n_ell):
            for i in range(self.n_z):
                for j in range(i, self.n_z):
                    ps[b, i, j] = ps[b, j, i] = d[a]
                    a += 1
            for i in range(self.n_z):
                ps[b, i, i] += self.shot_noise()
        return ps

    def nmodes(self):
        return np.array(n_modes(self.centres[:self.n_ell], self.widths[:self.n_ell], self.f_sky))

    def ntri(self, lattice=None):
        if lattice is not None:
            return np.asarray(lattice, np.float64)
        c, w = self.centres, self.widths
        return np.array([n_tri_closed(c[i], c[j], c[k], w[i], w[j], w[k], self.f_sky)
                         for (i, j, k, _) in self.tris], np.float64)

    def u_table(self):
        if self._U is None:
            ell = np.array(self.centres[:self.n_ell], np.float64)
            U = np.zeros((self.n_ell, self.n_chi, self.n_m))
            lib().or_clear_error()
            lib().or_tab_u(ct.byref(self.T), ct.c_int(self.n_ell), _p(ell), _p(U))
            self._check()
            self._U = (ell, U)
        return self._U

    # ---- covariance
    def cov1h_pairs(self, pairs):
        if self.n_sub > 1:
            return self.cov1h_avg_pairs(pairs)
        ell, U = self.u_table()
        pairs = np.ascontiguousarray(pairs, np.int64)
        out = np.zeros(len(pairs))
        zb = np.ascontiguousarray(self.rows["zbin"], np.int32)
        lb = np.ascontiguousarray(self.rows["lbin"], np.int32)
        lib().or_cov1h_pairs(ct.byref(self.T), _p(ell), _p(U), ct.c_double(self.omega),
                             _p(self.rows["kind"]), _p(lb), _p(zb), ct.c_int64(len(pairs)),
                             _p(pairs), _p(out))
        return out

    def gauss_pairs(self, pairs, ntri=None):
        ps = self.ps_table()
        nm = self.nmodes()
        nt = self.ntri(ntri)
        pairs = np.ascontiguousarray(pairs, np.int64)
        out = np.zeros(len(pairs))
        zb = np.ascontiguousarray(self.rows["zbin"], np.int32)
        lb = np.ascontiguousarray(self.rows["lbin"], np.int32)
        lib().or_gauss_pairs(ct.c_int(self.n_z), _p(ps), _p(nm), _p(nt), ct.c_double(self.omega),
                             _p(self.rows["kind"]), _p(lb), _p(zb), _p(self.rows["tri"]),
                             ct.c_int64(len(pairs)), _p(pairs), _p(out))
        return out

    def bfull(self):
        """Projected bispectrum of every triangle for every ordering of bins
        on its legs, [n_tri][n_z][n_z][n_z]: the data-vector value of the
        multiset of bins (the Limber kernels are symmetric in the bins)."""
        if getattr(self, "_bfull", None) is None:
            d, _ = self.data_vector()
            nz, nt = self.n_z, len(self.tris)
            val = {}
            for a in range(self.N):
                if self.rows["kind"][a] == 3:
                    val[(int(self.rows["tri"][a]), tuple(sorted(int(x) for x in self.rows["zbin"][a])))] = d[a]
            B = np.zeros((max(nt, 1), nz, nz, nz))
            for t in range(nt):
                for i in range(nz):
                    for j in range(nz):
                        for k in range(nz):
                            B[t, i, j, k] = val[(t, tuple(sorted((i, j, k))))]
            self._bfull = np.ascontiguousarray(B)
        return self._bfull

    def trispec(self, legs, z):
        """Projected one-halo trispectrum at four ell-bins and redshift bins."""
        ell, U = self.u_table()
        legs = np.ascontiguousarray(legs, np.int32)
        z = np.ascontiguousarray(z, np.int32)
        lib().or_trispec.restype = ct.c_double
        return lib().or_trispec(ct.byref(self.T), _p(ell), _p(U), _p(legs), _p(z))

    def ngins_pairs(self, pairs, rows=None):
        """The B.B, P.T and P.B in-survey terms (eqs. CovBB, Covpb) for the
        given (a, b) pairs of rows (default: the data-vector rows)."""
        rows = self.rows if rows is None else rows
        if self.n_sub > 1:
            raise ValueError("the in-survey B.B, P.T, P.B terms are not bin-averaged")
        ell, U = self.u_table()
        ps, nm, bf = self.ps_table(), self.nmodes(), self.bfull()
        pairs = np.ascontiguousarray(pairs, np.int64)
        out = np.zeros(len(pairs))
        lib().or_ngins_pairs(ct.byref(self.T), _p(ell), _p(U), ct.c_int(self.n_z), _p(ps), _p(nm), _p(bf),
                             _p(np.ascontiguousarray(rows["kind"], np.int32)),
                             _p(np.ascontiguousarray(rows["lbin"], np.int32)),
                             _p(np.ascontiguousarray(rows["zbin"], np.int32)),
                             _p(np.ascontiguousarray(rows["tri"], np.int32)), ct.c_int64(len(pairs)),
                             _p(pairs), _p(out))
        return out

    # ---- super-sample term resolved along the line of sight
    SIGMA_W_NODES = 16384

    def theta_sky(self):
        """Angular radius of the survey, Omega = 2 pi (1 - cos Theta) (the
        relation given after eq. PSest, Sec. 3.2.2)."""
        return math.acos(1.0 - self.omega / (2.0 * math.pi))

    def sigma_w2(self, n_eps=SIGMA_W_NODES):
        """sigma_W^2(chi_n) at every chi node (eq. Mask in the thin-shell
        limit, App. B; definition after eq. CovPP22)."""
        out = np.zeros(self.n_chi)
        lib().or_sigma_w2(ct.byref(self.T), ct.c_double(self.theta_sky()), ct.c_int(n_eps), _p(out))
        return out

    def ssc_chi_pairs(self, pairs, rows=None, sw=None):
        """The super-sample term of eq. WLSSCflatskyLimber with sigma_W^2(chi)
        for the given (a, b) pairs of rows (default: the data-vector rows)."""
        rows = self.rows if rows is None else rows
        sw = self.sigma_w2() if sw is None else np.ascontiguousarray(sw, np.float64)
        _, R = self.spectra()
        pairs = np.ascontiguousarray(pairs, np.int64)
        out = np.zeros(len(pairs))
        lib().or_ssc_chi_pairs(ct.byref(self.T), _p(sw), _p(R),
                               _p(np.ascontiguousarray(rows["kind"], np.int32)),
                               _p(np.ascontiguousarray(rows["zbin"], np.int32)),
                               _p(np.ascontiguousarray(rows["cfg"], np.int32)), ct.c_int64(len(pairs)),
                               _p(pairs), _p(out))
        return out

    def cov_pairs(self, pairs, ntri=None, ngins=False, ssc="rank1"):
        """Covariance entries C[a, b] for the given (a, b) pairs: Gaussian +
        one-halo + super-sample term (+ the B.B, P.T and P.B terms when ngins
        is set).  ssc="rank1": sigma_b^2 r r^T (one coherent long mode);
        ssc="chi": the line-of-sight form with sigma_W^2(chi)."""
        pairs = np.ascontiguousarray(pairs, np.int64)
        if ssc == "chi":
            sscv = self.ssc_chi_pairs(pairs)
        else:
            _, r = self.data_vector()
            sscv = float(self.cfg["sigma_b2"]) * r[pairs[:, 0]] * r[pairs[:, 1]]
        out = self.gauss_pairs(pairs, ntri) + self.cov1h_pairs(pairs) + sscv
        if ngins:
            out = out + self.ngins_pairs(pairs)
        return out

    def covariance(self, ntri=None, ngins=False, ssc="rank1"):
        """Full joint covariance C^D (eq. eq:SN2) on the lower triangle,
        mirrored (+ the B.B, P.T and P.B terms when ngins is set; ssc as in
        cov_pairs)."""
        canon, reps = canonical_rows(self.rows)
        nc = len(reps)
        ell, U = self.u_table()
        kind = np.ascontiguousarray(self.rows["kind"][reps], np.int32)
        lb = np.ascontiguousarray(self.rows["lbin"][reps], np.int32)
        zb = np.ascontiguousarray(self.rows["zbin"][reps], np.int32)
        c1h = np.zeros((nc, nc))
        if self.n_sub > 1:
            ii, jj = np.tril_indices(nc)
            c1h[ii, jj] = self.cov1h_avg_pairs(np.stack([reps[ii], reps[jj]], 1))
        else:
            lib().or_cov1h_canon(ct.byref(self.T), _p(ell), _p(U), ct.c_double(self.omega), ct.c_int(nc),
                                 _p(kind), _p(lb), _p(zb), _p(c1h))
        _, r = self.data_vector()
        ps = self.ps_table()
        nm = self.nmodes()
        nt = self.ntri(ntri)
        C = np.zeros((self.N, self.N))
        zbf = np.ascontiguousarray(self.rows["zbin"], np.int32)
        lbf = np.ascontiguousarray(self.rows["lbin"], np.int32)
        lib().or_cov_full(ct.c_int(self.N), _p(c1h), ct.c_int(nc), _p(canon), ct.c_int(self.n_z),
                          _p(ps), _p(nm), _p(nt), ct.c_double(self.omega), _p(self.rows["kind"]),
                          _p(lbf), _p(zbf), _p(self.rows["tri"]), _p(r),
                          ct.c_double(float(self.cfg["sigma_b2"]) if ssc != "chi" else 0.0), _p(C))
        extra = []
        if ngins:
            extra.append(self.ngins_pairs)
        if ssc == "chi":
            extra.append(self.ssc_chi_pairs)
        if extra:
            ii, jj = np.tril_indices(self.N)
            for f in extra:
                v = f(np.stack([ii, jj], 1))
                C[ii, jj] += v
                C[jj[ii != jj], ii[ii != jj]] += v[ii != jj]
        return C

    @staticmethod
    def snr2(C, d):
        """(S/N)^2 = D^T C^-1 D (eq. SNprim) by Cholesky-Banachiewicz."""
        C = np.ascontiguousarray(C, np.float64)
        d = np.ascontiguousarray(d, np.float64)
        out = ct.c_double(0.0)
        rc = lib().or_snr2(ct.c_int(len(d)), _p(C), _p(d), ct.byref(out))
        if rc == -1:
            raise np.linalg.LinAlgError("covariance is not positive definite")
        if rc != 0:
            raise MemoryError("oracle S/N allocation failed")
        return out.value

    @staticmethod
    def chol_y(C, d):
        """y = L^-1 d with C = L L^T (the forward substitution of eq. SNprim)."""
        C = np.ascontiguousarray(C, np.float64)
        d = np.ascontiguousarray(d, np.float64)
        y = np.zeros(len(d))
        rc = lib().or_chol_y(ct.c_int(len(d)), _p(C), _p(d), _p(y))
        if rc == -1:
            raise np.linalg.LinAlgError("covariance is not positive definite")
        if rc != 0:
            raise MemoryError("oracle allocation failed")
        return y

    def lmax_order(self):
        """Data-vector rows ordered by the largest ell-bin among their legs
        (stable), and the number of rows whose largest bin is <= b for each
        bin b.  The leading rows up to bin b are the data vector cut at an
        ell_max between bins b and b + 1 (eq. eq:SN)."""
        top = np.where(self.rows["kind"] == 2, self.rows["lbin"][:, 0], np.max(self.rows["lbin"], axis=1))
        order = np.argsort(top, kind="stable")
        ends = np.array([np.count_nonzero(top <= b) for b in range(self.n_ell)], np.int64)
        return order, ends

    def snr2_lmax(self, C, d):
        """(S/N)^2 of the data vector cut at every ell_max (eq. eq:SN): the
        covariance of a cut vector is a principal submatrix of C, so with the
        rows in lmax_order one Cholesky gives all cuts as prefix sums of y^2."""
        order, ends = self.lmax_order()
        y = self.chol_y(np.asarray(C)[np.ix_(order, order)], np.asarray(d)[order])
        cs = np.cumsum(y * y)
        return cs[ends - 1]

    @staticmethod
    def pca(C, d, vectors=True):
        """Principal components of the covariance (Sec. 6): C = sum_a lambda_a
        S_a S_a^T (eq. SNPCA), the new observables D^_a = S_a . D (eq. NewObs)
        and their (S/N)^2_a = D^_a^2 / lambda_a (eq. SNperEign).  Returns the
        eigenvalues ascending, the (S/N)^2 of each mode in that order, the
        cumulative (S/N)^2 over the modes taken by decreasing (S/N)^2 (eq.
        CumulSN in the order of the paper's second PCA figure) and, with
        vectors, S with row a the unit eigenvector of mode a (sign: its
        largest entry in magnitude is positive).

        The eigenvalues span tens of decades, and a symmetric eigensolver
        resolves only those above about 1e-16 of the largest.  So the
        eigenpairs come from LAPACK's preconditioned Jacobi SVD (dgejsv),
        which keeps relative accuracy on graded matrices: with Delta the
        powers of two that bring the diagonal of Delta^-1 C Delta^-1 to
        [1, 4) and Delta^-1 C Delta^-1 = L L^T, C = G^T G for G = L^T Delta,
        whose singular values are sqrt(lambda) and whose right singular
        vectors are the eigenvectors of C."""
        from scipy.linalg import lapack
        C = np.asarray(C, np.float64)
        d = np.asarray(d, np.float64)
        delta = np.ldexp(1.0, np.frexp(np.sqrt(np.diag(C)))[1])
        L = np.linalg.cholesky(C / np.outer(delta, delta))
        G = np.ascontiguousarray(L.T * delta[None, :])
        sva, _, v, work, _, info = lapack.dgejsv(G, joba=2, jobu=3, jobv=0)
        if info != 0:
            raise np.linalg.LinAlgError("dgejsv failed (%d)" % info)
        lam = (sva * (work[0] / work[1])) ** 2
        S = v.T.copy()
        o = np.argsort(lam, kind="stable")
        lam, S = lam[o], S[o]
        snr2 = (S @ d) ** 2 / lam
        cum = np.cumsum(np.sort(snr2)[::-1])
        if not vectors:
            return lam, snr2, cum
        big = np.argmax(np.abs(S), axis=1)
        S *= np.sign(S[np.arange(len(S)), big])[:, None]
        return lam, snr2, cum, S

    def run(self, ntri=None, ngins=False, ssc="rank1"):
        d, r = self.data_vector()
        C = self.covariance(ntri, ngins, ssc)
        return dict(d=d, r=r, C=C, snr2=self.snr2(C, d))

    # ---- scalar pieces for pins
    def halo_I(self, mu, beta, ks):
        ks = np.ascontiguousarray(ks, np.float64)
        return lib().or_halo_I(ct.byref(self.T), ct.c_int(mu), ct.c_int(beta), _p(ks))

    def spectrum(self, n, ks):
        ks = np.ascontiguousarray(ks, np.float64)
        X = ct.c_double(); R = ct.c_double()
        kind = 2 if len(ks) == 1 else 3
        lib().or_spectrum(ct.byref(self.T), ct.c_int(n), ct.c_int(kind), _p(ks), ct.byref(X), ct.byref(R))
        return X.value, R.value


def interp(kgrid, row, k):
    kgrid = np.ascontiguousarray(kgrid, np.float64)
    row = np.ascontiguousarray(row, np.float64)
    lib().or_interp.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_double]
    return lib().or_interp(_p(kgrid), _p(row), len(kgrid), float(k))


def neff(kgrid, row, k):
    kgrid = np.ascontiguousarray(kgrid, np.float64)
    row = np.ascontiguousarray(row, np.float64)
    lib().or_neff.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_double]
    return lib().or_neff(_p(kgrid), _p(row), len(kgrid), float(k))


def F2(ki, kj, kl):
    return lib().or_F2(ki, kj, kl)
