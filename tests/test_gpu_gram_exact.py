"""The one-halo Gram kernels (eq. General1h: the one-halo covariance of the
distinct rows is A A^T / Omega over the flattened (chi, M) axis) on integer
factors, through wlc_gram.  With |hi| <= 8, |lo| <= 4 every bf16 operand,
every product and every FP32 partial sum is an exact integer below 2^24, so
whatever the summation order the result must equal the integer product bit
for bit: hi hi^T for one product, hi hi^T + hi lo^T + lo hi^T for the split
product (lo lo^T dropped).

The shapes cover one and several 256-row tiles, padding rows and columns, and
split-K slices whose stage counts (32 columns each) take every residue mod 3
of the one-product ring (three stage buffers) and both parities of the split
product's two stage buffers, as well as slices too short for the ring's
steady state (two stages; with panel extents, slices of one stage and empty
ones).  With panel extents, the factors hold NaN past each
panel's extent: a product that read a column it must skip would not be
finite."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# (n, k): stage counts per slice with the split-K choice of the library (the
# same for every bf16 mode; the one-product ring has three stage buffers, the
# split product two)
CASES = [
    (256, 64),      # one tile, one slice of 2 stages
    (256, 2048),    # one slice of 64 stages (1 mod 3, even)
    (200, 4000),    # padding rows and columns (k_pad 4032): one slice of 126 (0 mod 3)
    (1280, 32768),  # 15 tiles: four slices of 256 (1 mod 3)
    (1280, 33024),  # four slices of 258 (0 mod 3)
    (1100, 34816),  # padding rows: four slices of 272 (2 mod 3)
    (768, 8320),    # 6 tiles: four slices of 65 (2 mod 3, odd)
]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _bf16_bits(x):
    """bf16 bit patterns of small integers (exact)."""
    return (np.asarray(x, np.float32).view(np.uint32) >> 16).astype(np.uint16)


def _kblocked(bits, n_pad, k_pad):
    """The k-blocked layout: element (r, c) at ((c / 32) n_pad + r) 32 + c % 32."""
    n, k = bits.shape
    full = np.zeros((n_pad, k_pad), np.uint16)
    full[:n, :k] = bits
    return np.ascontiguousarray(full.reshape(n_pad, k_pad // 32, 32).transpose(1, 0, 2)).reshape(-1)


@pytest.fixture(scope="module")
def wl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1812_07437_amd import wlcov
    return wlcov


@pytest.fixture(scope="module", params=CASES, ids=["n%d_k%d" % c for c in CASES])
def case(request, wl):
    n, k = request.param
    rng = np.random.default_rng(20191218 + n + k)
    hi = rng.integers(-8, 9, size=(n, k)).astype(np.float64)
    lo = rng.integers(-4, 5, size=(n, k)).astype(np.float64)
    n_pad, k_pad = -(-n // 256) * 256, -(-k // 64) * 64
    dev = torch.device("cuda:0")
    a_hi = torch.from_numpy(_kblocked(_bf16_bits(hi), n_pad, k_pad).view(np.int16)).to(dev)
    a_lo = torch.from_numpy(_kblocked(_bf16_bits(lo), n_pad, k_pad).view(np.int16)).to(dev)
    hh = np.zeros((n_pad, n_pad))
    hl = np.zeros((n_pad, n_pad))
    hh[:n, :n] = hi @ hi.T  # integers below 2^53: exact in float64 whatever the order
    hl[:n, :n] = hi @ lo.T
    return dict(n=n, k=k, n_pad=n_pad, a_hi=a_hi, a_lo=a_lo, hh=hh, split=hh + hl + hl.T)


def _run(wl, c, precision, panel_f=None, lim=0.0):
    n, k, n_pad = c["n"], c["k"], c["n_pad"]
    ext = c.get("ext")
    dev = torch.device("cuda:0")
    ws_b = wl.wlc_gram_ws_bytes(precision, n, k)
    ws = torch.empty(max(ws_b, 256), dtype=torch.uint8, device=dev)
    g = torch.full((n_pad, n_pad), float("nan"), dtype=torch.float32, device=dev)
    pf = None if panel_f is None else torch.as_tensor(panel_f, dtype=torch.float64).to(dev)
    pe = None if ext is None else torch.as_tensor(ext, dtype=torch.int32).to(dev)
    stream = torch.cuda.current_stream()
    _say("case gram exact n=%d k=%d %s ext %s" % (n, k, precision, ext))
    wl.wlc_gram(precision, n, k, wl._ptr(c["a_hi"]), wl._ptr(c["a_lo"]), wl._ptr(pf) if pf is not None else None,
                lim, wl._ptr(g), wl._ptr(ws), wl._stream_handle(stream),
                panel_ext=wl._ptr(pe) if pe is not None else None)
    torch.cuda.synchronize()
    return g.cpu().numpy().astype(np.float64)


def _check_tiles(G, want_of_tile, n_pad):
    """Every entry i >= j of every 256-tile I >= J (above the diagonal of a
    diagonal tile the split-K slices are not summed)."""
    nt = n_pad // 256
    low = np.tril(np.ones((256, 256), bool))
    for I in range(nt):
        for J in range(I + 1):
            s = np.s_[256 * I:256 * I + 256, 256 * J:256 * J + 256]
            got, want = G[s], want_of_tile(I, J)[s]
            if I == J:
                got, want = got[low], want[low]
            assert np.array_equal(got, want), (I, J, float(np.max(np.abs(got - want))))


def test_one_product_exact(wl, case):
    G = _run(wl, case, "bf16")
    _check_tiles(G, lambda I, J: case["hh"], case["n_pad"])


def test_split_product_exact(wl, case):
    G = _run(wl, case, "bf16x3")
    _check_tiles(G, lambda I, J: case["split"], case["n_pad"])


def test_per_tile_choice_exact(wl, case):
    """Panels alternate between F = 0.1 and F = 1 with the limit 0.5: the
    tiles between two odd panels take the split product, the others one."""
    nt = case["n_pad"] // 256
    F = np.array([1.0 if I % 2 else 0.1 for I in range(nt)])
    G = _run(wl, case, "bf16_auto", panel_f=F, lim=0.5)
    _check_tiles(G, lambda I, J: case["split"] if F[I] * F[J] > 0.5 else case["hh"], case["n_pad"])


def test_upper_tiles_untouched(wl, case):
    """Only the tiles I >= J are written."""
    if case["n_pad"] == 256:
        pytest.skip("one tile")
    G = _run(wl, case, "bf16")
    assert np.isnan(G[0:256, 256:512]).all()


# Panel extents: the rows of panel I are zero from column 32 ext_I on, and the
# k-blocked factors hold NaN there, which the product must not read.
EXT_CASES = [(200, 4000), (1280, 33024), (1100, 34816)]
BF16_NAN = 0x7FC0


def _extents(nt, nb):
    """Full, about half, one block, none (a panel of zeros), all but five."""
    if nt == 1:
        return [nb // 2 + 3]
    pattern = [nb, nb // 2 + 3, 1, 0, nb - 5]
    return [pattern[I % len(pattern)] for I in range(nt)]


@pytest.fixture(scope="module", params=EXT_CASES, ids=["n%d_k%d" % c for c in EXT_CASES])
def ext_case(request, wl):
    n, k = request.param
    rng = np.random.default_rng(20190220 + n + k)
    n_pad, k_pad = -(-n // 256) * 256, -(-k // 64) * 64
    nt, nb = n_pad // 256, k_pad // 32
    ext = _extents(nt, nb)
    hi = rng.integers(-8, 9, size=(n, k)).astype(np.float64)
    lo = rng.integers(-4, 5, size=(n, k)).astype(np.float64)
    for I in range(nt):
        hi[256 * I:256 * I + 256, 32 * ext[I]:] = 0.0
        lo[256 * I:256 * I + 256, 32 * ext[I]:] = 0.0

    def blocked(x):
        b = _kblocked(_bf16_bits(x), n_pad, k_pad).reshape(nb, n_pad, 32)
        for I in range(nt):
            b[ext[I]:, 256 * I:256 * I + 256, :] = BF16_NAN
        return b.reshape(-1)

    dev = torch.device("cuda:0")
    a_hi = torch.from_numpy(blocked(hi).view(np.int16)).to(dev)
    a_lo = torch.from_numpy(blocked(lo).view(np.int16)).to(dev)
    hh = np.zeros((n_pad, n_pad))
    hl = np.zeros((n_pad, n_pad))
    hh[:n, :n] = hi @ hi.T
    hl[:n, :n] = hi @ lo.T
    return dict(n=n, k=k, n_pad=n_pad, ext=ext, a_hi=a_hi, a_lo=a_lo, hh=hh, split=hh + hl + hl.T)


def test_extent_one_product_exact(wl, ext_case):
    G = _run(wl, ext_case, "bf16")
    _check_tiles(G, lambda I, J: ext_case["hh"], ext_case["n_pad"])


def test_extent_split_product_exact(wl, ext_case):
    G = _run(wl, ext_case, "bf16x3")
    _check_tiles(G, lambda I, J: ext_case["split"], ext_case["n_pad"])


def test_extent_per_tile_choice_exact(wl, ext_case):
    nt = ext_case["n_pad"] // 256
    F = np.array([1.0 if I % 2 else 0.1 for I in range(nt)])
    G = _run(wl, ext_case, "bf16_auto", panel_f=F, lim=0.5)
    _check_tiles(G, lambda I, J: ext_case["split"] if F[I] * F[J] > 0.5 else ext_case["hh"], ext_case["n_pad"])
