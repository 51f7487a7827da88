"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these compare the oracle with itself: each checks a hand-worked
example, a closed form, an invariant, a public standard's worked example, a
brute force over tiny inputs, or an independent textbook formulation.
"""
from __future__ import annotations

import heapq
import itertools
import math
import os

import numpy as np
import pytest

import archive_util as au

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_golden(name):
    """Parse a golden fixture: '#' comments, then 'key: values' lines."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, v = line.split(":", 1)
            out[k.strip()] = [int(t) for t in v.split()]
    return out


# --------------------------------------------------------------------------
# Lorenzo predictor (Sec. 3.1.2; padding layer Sec. 3.1.1)
# --------------------------------------------------------------------------

def test_lorenzo_worked_examples(orc):
    g = load_golden("lorenzo_worked.txt")
    d1 = np.array(g["dq_1d"], np.int32)
    assert orc.lorenzo_delta(d1).tolist() == g["delta_1d"]
    d2 = np.array(g["dq_2d"], np.int32).reshape(3, 3)
    assert orc.lorenzo_delta(d2).ravel().tolist() == g["delta_2d"]
    d3 = np.array(g["dq_3d"], np.int32).reshape(2, 2, 2)
    assert orc.lorenzo_delta(d3).ravel().tolist() == g["delta_3d"]


@pytest.mark.parametrize("shape,block", [((70,), (32,)), ((37, 21), (16, 16)), ((11, 19, 13), (8, 8, 8))])
def test_lorenzo_constant_field_unit_weight(orc, shape, block):
    """Coefficients sum to 1: a constant field is predicted exactly except at
    each block's first point, whose neighbours are all padding (value 0)."""
    c = 12345
    d = np.full(shape, c, np.int32)
    delta = orc.lorenzo_delta(d)
    first = np.ones(shape, bool)
    for ax, b in enumerate(block):
        idx = np.arange(shape[ax]) % b == 0
        sh = [1] * len(shape)
        sh[ax] = shape[ax]
        first &= idx.reshape(sh)
    assert np.all(delta[first] == c)
    assert np.all(delta[~first] == 0)


def test_lorenzo_2d_affine_and_outer_layer(orc):
    """2D: for d = a + b*x + c*y the predictor is exact inside a block; on a
    block's first row/column it falls back to 1D Lorenzo along the other
    axis (padding layer is 0)."""
    ny, nx = 40, 37
    a, b, c = 7, 3, -5
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    d = (a + b * x + c * y).astype(np.int32)
    delta = orc.lorenzo_delta(d)
    iy, ix = y % 16, x % 16
    interior = (iy > 0) & (ix > 0)
    assert np.all(delta[interior] == 0)
    assert np.all(delta[(iy == 0) & (ix > 0)] == b)
    assert np.all(delta[(iy > 0) & (ix == 0)] == c)
    corner = (iy == 0) & (ix == 0)
    assert np.all(delta[corner] == d[corner])


def test_lorenzo_3d_exact_on_pairwise_sums(orc):
    """3D 1-layer Lorenzo annihilates g(y,x) + h(z,y) + k(z,x) inside a block
    (the mixed third difference of a sum of two-variable functions is 0)."""
    rng = np.random.default_rng(5)
    nz, ny, nx = 17, 12, 19
    g = rng.integers(-1000, 1000, (ny, nx))
    h = rng.integers(-1000, 1000, (nz, ny))
    k = rng.integers(-1000, 1000, (nz, nx))
    d = (g[None, :, :] + h[:, :, None] + k[:, None, :]).astype(np.int32)
    delta = orc.lorenzo_delta(d)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    interior = (z % 8 > 0) & (y % 8 > 0) & (x % 8 > 0)
    assert np.all(delta[interior] == 0)
    assert np.any(delta[~interior] != 0)


def _blockwise_cumsum_inverse(delta, block):
    """Independent inverse: inside each block, the Lorenzo map is the mixed
    backward difference, so its inverse is a prefix sum along every axis
    (mod 2^32).  Written with numpy cumsum per block."""
    out = np.empty_like(delta, dtype=np.int64)
    shape = delta.shape
    ranges = [range(0, s, b) for s, b in zip(shape, block)]
    for starts in itertools.product(*ranges):
        sl = tuple(slice(s0, min(s0 + b, n)) for s0, b, n in zip(starts, block, shape))
        v = delta[sl].astype(np.int64)
        for ax in range(delta.ndim):
            v = np.cumsum(v, axis=ax)
        out[sl] = v
    return (out & 0xFFFFFFFF).astype(np.uint32).view(np.int32)


@pytest.mark.parametrize("shape,block", [((100,), (32,)), ((35, 18), (16, 16)), ((9, 17, 10), (8, 8, 8))])
def test_lorenzo_inverse_equals_prefix_sums_with_wraparound(orc, shape, block):
    rng = np.random.default_rng(11)
    dq = rng.integers(-2**31, 2**31, size=shape, dtype=np.int64).astype(np.int32)
    delta = orc.lorenzo_delta(dq)
    assert np.array_equal(_blockwise_cumsum_inverse(delta, block), dq)
    assert np.array_equal(orc.lorenzo_reconstruct(delta), dq)


# --------------------------------------------------------------------------
# 2-layer Lorenzo predictor (the generalized predictor of Sec. 3.1.2, n = 2)
# --------------------------------------------------------------------------

def test_lorenzo2_worked_examples(orc):
    g = load_golden("lorenzo2_worked.txt")
    assert orc.lorenzo_delta(np.array(g["dq_1d"], np.int32), 2).tolist() == g["delta_1d"]
    d2 = np.array(g["dq_2d"], np.int32).reshape(3, 3)
    assert orc.lorenzo_delta(d2, 2).ravel().tolist() == g["delta_2d"]
    d3 = np.array(g["dq_3d"], np.int32).reshape(2, 2, 2)
    assert orc.lorenzo_delta(d3, 2).ravel().tolist() == g["delta_3d"]


@pytest.mark.parametrize("shape,block", [((70,), (32,)), ((37, 21), (16, 16)), ((11, 19, 13), (8, 8, 8))])
def test_lorenzo2_constant_field_closed_form(orc, shape, block):
    """Unit weight: a constant c gives delta = c * prod_axes a(i mod b) with
    a(0) = 1, a(1) = -1, a(>=2) = 0 ((1 - S)^2 of a step that starts at the
    block's padding)."""
    c = 777
    delta = orc.lorenzo_delta(np.full(shape, c, np.int32), 2)
    want = np.full(shape, c, np.int64)
    for ax, b in enumerate(block):
        i = np.arange(shape[ax]) % b
        a = np.where(i == 0, 1, np.where(i == 1, -1, 0))
        sh = [1] * len(shape)
        sh[ax] = shape[ax]
        want = want * a.reshape(sh)
    assert np.array_equal(delta.astype(np.int64), want)


def test_lorenzo2_annihilates_fields_linear_along_an_axis(orc):
    """(1 - S)^2 along an axis annihilates anything linear along it, whatever
    the dependence on the other axes: delta = 0 at points two or more steps
    into the block along that axis."""
    rng = np.random.default_rng(21)
    x = np.arange(90)
    d1 = (17 + 5 * x).astype(np.int32)
    assert np.all(orc.lorenzo_delta(d1, 2)[x % 32 >= 2] == 0)
    ny, nx = 33, 40
    g, h = rng.integers(-99, 99, ny), rng.integers(-99, 99, ny)
    d2 = (g[:, None] + h[:, None] * np.arange(nx)[None, :]).astype(np.int32)     # linear in x
    assert np.all(orc.lorenzo_delta(d2, 2)[:, np.arange(nx) % 16 >= 2] == 0)
    d2t = np.ascontiguousarray(d2.T[:ny, :]) if nx >= ny else None                   # linear in y
    assert np.all(orc.lorenzo_delta(d2t, 2)[np.arange(ny) % 16 >= 2, :] == 0)
    nz, ny3, nx3 = 19, 10, 11
    gg, hh = rng.integers(-99, 99, (ny3, nx3)), rng.integers(-99, 99, (ny3, nx3))
    d3 = (gg[None] + hh[None] * np.arange(nz)[:, None, None]).astype(np.int32)      # linear in z
    assert np.all(orc.lorenzo_delta(d3, 2)[np.arange(nz) % 8 >= 2] == 0)
    assert np.any(orc.lorenzo_delta(d3, 2) != 0)


@pytest.mark.parametrize("shape", [(100,), (35, 18), (9, 17, 10)])
def test_lorenzo2_is_the_1layer_map_twice(orc, shape):
    """The binomial 2-layer form equals the explicit 1-layer predictor's
    delta map applied twice (each with the zero padding), mod 2^32."""
    rng = np.random.default_rng(len(shape))
    d = rng.integers(-2**31, 2**31, size=shape, dtype=np.int64).astype(np.int32)
    assert np.array_equal(orc.lorenzo_delta(d, 2), orc.lorenzo_delta(orc.lorenzo_delta(d)))


@pytest.mark.parametrize("shape,block", [((100,), (32,)), ((35, 18), (16, 16)), ((9, 17, 10), (8, 8, 8))])
def test_lorenzo2_inverse_is_prefix_sums_twice_with_wraparound(orc, shape, block):
    rng = np.random.default_rng(13)
    dq = rng.integers(-2**31, 2**31, size=shape, dtype=np.int64).astype(np.int32)
    delta = orc.lorenzo_delta(dq, 2)
    assert np.array_equal(_blockwise_cumsum_inverse(_blockwise_cumsum_inverse(delta, block), block), dq)
    assert np.array_equal(orc.lorenzo_reconstruct(delta, 2), dq)


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_compress2_round_trip_within_bound(orc, ndim):
    """Whole pipeline with the 2-layer predictor: the header records it, the
    field comes back within the bound, and on a smooth field most points
    need no outlier."""
    from synth import fields
    x = {1: lambda: fields.particles1d(20000, seed=1, shuffle_block=256),
         2: lambda: fields.fourier2d((60, 90), seed=2),
         3: lambda: fields.hurricane3d((20, 24, 28), seed=3)}[ndim]()
    arc = orc.compress(x, 1e-3, orc.EB_VALREL, layers=2)
    assert int(arc[117]) == 1
    assert int(orc.compress(x, 1e-3, orc.EB_VALREL)[117]) == 0
    y = orc.decompress(arc)
    eb_abs = au.header(arc)["eb_abs"]
    assert np.all(np.abs(x.astype(np.float64) - y.astype(np.float64)) <= eb_abs)
    # same prequantized values as the 1-layer archive: the floats agree
    assert np.array_equal(y.view(np.uint32), orc.decompress(orc.compress(x, 1e-3, orc.EB_VALREL)).view(np.uint32))


# --------------------------------------------------------------------------
# Prequantization (Sec. 3.1.2) and the error bound
# --------------------------------------------------------------------------

def test_eb_params_closed_forms(orc):
    e, h, r = orc.eb_params(0, 2.0 ** -11)
    assert e == 2.0 ** -11 and h == np.float32(2.0 ** -10) and r == np.float32(2.0 ** 10)
    e, h, r = orc.eb_params(1, 1e-4, np.float32(-3.0), np.float32(5.0), 10)
    assert e == 1e-4 * 8.0
    assert h == np.float32(2 * 8e-4) and r == np.float32(1.0 / (2 * 8e-4))
    # constant field or no finite values: range taken as 1
    assert orc.eb_params(1, 1e-3, np.float32(2.0), np.float32(2.0), 5)[0] == 1e-3
    assert orc.eb_params(1, 1e-3, 0.0, 0.0, 0)[0] == 1e-3
    for bad in (0.0, -1.0, float("nan"), float("inf"), 1e-300, 1e300):
        with pytest.raises(orc.OracleError):
            orc.eb_params(0, bad)


def test_value_range_total_order(orc):
    x = np.array([np.nan, 0.0, -0.0, np.inf, -np.inf, 1.5, -2.5], np.float32)
    lo, hi, n = orc.value_range(x)
    assert (lo, hi, n) == (np.float32(-2.5), np.float32(1.5), 4)
    lo, hi, n = orc.value_range(np.array([0.0, -0.0, 0.0], np.float32))
    assert np.signbit(lo) and not np.signbit(hi)


def test_prequant_round_half_even_exact_grid(orc):
    """With h = 2^-10 every product is exact, so d° is round(d / 2eb) with
    ties to even, and the posterror |d - 2eb d°| never exceeds eb."""
    r = np.float32(1024.0)
    k = np.arange(-40, 41)
    x = (k / 2.0 / 1024.0).astype(np.float32)          # half-integers of the grid
    dq = orc.prequant(x, r)
    expect = np.array([int(round(v / 2.0)) for v in k])  # Python round: ties to even
    assert dq.tolist() == expect.tolist()
    assert np.all(np.abs(x.astype(np.float64) - dq * (1 / 1024.0)) <= 0.5 / 1024.0)
    special = np.array([np.nan, np.inf, -np.inf, 3e9 / 1024.0], np.float32)
    assert orc.prequant(special, r).tolist() == [0, 0, 0, 0]


# --------------------------------------------------------------------------
# Histogram (Sec. 3.2.1)
# --------------------------------------------------------------------------

def test_histogram_is_bincount(orc):
    from synth import fields
    x = fields.hurricane3d((20, 33, 41), seed=7)
    dq, codes, freq, _ = orc.stages(x, 1e-3)
    assert freq.sum() == x.size
    assert np.array_equal(freq, np.bincount(codes, minlength=1024).astype(np.uint64))


# --------------------------------------------------------------------------
# Huffman lengths (Sec. 3.2.2)
# --------------------------------------------------------------------------

def _brute_force_min_cost(freq):
    """Minimum of sum f_i l_i over all length vectors with Kraft sum <= 1."""
    n = len(freq)
    best = None
    for ls in itertools.product(range(1, n), repeat=n):
        if sum(2.0 ** -l for l in ls) <= 1.0 + 1e-12:
            c = sum(f * l for f, l in zip(freq, ls))
            best = c if best is None else min(best, c)
    return best


def _heap_huffman_cost(freq):
    """Textbook heap Huffman: cost = sum of all merged weights."""
    h = [f for f in freq if f > 0]
    if len(h) == 1:
        return h[0]
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a = heapq.heappop(h)
        b = heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


@pytest.mark.parametrize("seed", range(12))
def test_huffman_optimal_by_brute_force(orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 7))
    freq = rng.integers(1, 50, n).tolist()
    lens = orc.huffman_lengths(freq).astype(int)
    cost = sum(f * l for f, l in zip(freq, lens))
    assert cost == _brute_force_min_cost(freq)
    assert sum(2.0 ** -int(l) for l in lens) == 1.0      # Kraft equality


@pytest.mark.parametrize("seed", range(6))
def test_huffman_cost_matches_heap_and_entropy(orc, seed):
    rng = np.random.default_rng(100 + seed)
    freq = np.zeros(1024, np.uint64)
    used = rng.choice(1024, size=int(rng.integers(2, 1024)), replace=False)
    freq[used] = rng.geometric(0.01, size=used.size).astype(np.uint64)
    lens = orc.huffman_lengths(freq).astype(np.int64)
    assert np.all((lens > 0) == (freq > 0))
    cost = int((lens * freq.astype(np.int64)).sum())
    assert cost == _heap_huffman_cost(freq.astype(np.int64).tolist())
    f = freq[freq > 0].astype(np.float64)
    p = f / f.sum()
    H = -(p * np.log2(p)).sum()
    assert f.sum() * H <= cost + 1e-6 < f.sum() * (H + 1)
    assert math.isclose(sum(2.0 ** -int(l) for l in lens[lens > 0]), 1.0)


def test_huffman_tie_rules_pinned():
    """Hand-worked tie cases (fixture explains each)."""
    import oracle
    g = load_golden("huffman_ties.txt")
    assert oracle.huffman_lengths(g["freq_a"]).tolist() == g["len_a"]
    assert oracle.huffman_lengths(g["freq_b"]).tolist() == g["len_b"]
    assert oracle.huffman_lengths(g["freq_c"]).tolist() == g["len_c"]
    assert oracle.huffman_lengths(g["freq_d"]).tolist() == g["len_d"]


# --------------------------------------------------------------------------
# Canonical codebook (Sec. 3.2.3)
# --------------------------------------------------------------------------

def test_canonical_codes_rfc1951_example(orc):
    g = load_golden("canonical_rfc1951.txt")
    codes = orc.canonical_codes(g["lengths"])
    assert codes.tolist() == g["codes"]


def test_canonical_codes_prefix_free_and_ordered(orc):
    rng = np.random.default_rng(3)
    freq = rng.integers(0, 1000, 300).astype(np.uint64)
    lens = orc.huffman_lengths(freq)
    codes = orc.canonical_codes(lens)
    words = [format(int(c), "0%db" % l) for c, l in zip(codes, lens) if l]
    for a, b in itertools.combinations(words, 2):
        assert not a.startswith(b) and not b.startswith(a)
    # canonical order: sorting by (length, symbol) sorts the code values
    order = sorted((int(l), s) for s, l in enumerate(lens) if l)
    vals = [int(codes[s]) << (64 - l) for l, s in order]
    assert vals == sorted(vals)


# --------------------------------------------------------------------------
# Bitstream, tables, archive (Sec. 3.2.4)
# --------------------------------------------------------------------------

def _decode_all(stream_bits, lens):
    """Independent prefix-code decoder: greedy match against a dict."""
    import oracle
    codes = oracle.canonical_codes(lens)
    table = {format(int(c), "0%db" % l): s for s, (c, l) in enumerate(zip(codes, lens)) if l}
    out, cur = [], ""
    for b in stream_bits:
        cur += "1" if b else "0"
        if cur in table:
            out.append(table[cur])
            cur = ""
    assert cur == ""
    return out


def test_bitstream_and_tables(orc):
    from synth import fields
    x = fields.fourier2d((45, 70), seed=4)
    arc = orc.compress(x, 1e-4, sub_size=32, chunk_subs=2)
    s = au.sections(arc)
    h = s["header"]
    _, codes, freq, _ = orc.stages(x, 1e-4)
    lens = s["lengths"].astype(np.int64)
    assert h["total_bits"] == int((freq.astype(np.int64) * lens).sum())
    bits = au.stream_bits(s["stream"], h["total_bits"])
    assert _decode_all(bits, s["lengths"]) == codes.tolist()
    # trailing pad bits of the last word are zero
    if h["total_bits"] % 32:
        assert int(s["stream"][-1]) & ((1 << (32 - h["total_bits"] % 32)) - 1) == 0
    # subchunk entries sum to the stream; chunk entries are their prefix sums
    assert int(s["subs"].astype(np.int64).sum()) == h["total_bits"]
    pref = np.concatenate([[0], np.cumsum(s["subs"].astype(np.int64))])
    assert s["chunks"].tolist() == pref[::h["chunk_subs"]][:len(s["chunks"])].tolist()
    # the stream and subchunk table do not depend on the chunk grouping
    for c in (1, 4, 64):
        s2 = au.sections(orc.compress(x, 1e-4, sub_size=32, chunk_subs=c))
        assert np.array_equal(s2["stream"], s["stream"])
        assert np.array_equal(s2["subs"], s["subs"])


def test_codes_and_outliers_round_trip_losslessly(orc):
    """Postquantization adds no error: the decoder recovers every d° exactly,
    so each non-patched output equals fl32(d°) * h computed by numpy."""
    from synth import fields
    x = fields.hurricane3d((21, 30, 26), seed=9)
    x[3, 4, 5] = 1e4      # forces outliers around it
    arc = orc.compress(x, 1e-4)
    s = au.sections(arc)
    h = s["header"]
    dq, codes, _, _ = orc.stages(x, 1e-4)
    y = orc.decompress(arc)
    hf = np.array([h["h_bits"]], np.uint32).view(np.float32)[0]
    expect = dq.astype(np.float32) * hf
    patched = np.zeros(x.size, bool)
    keys = s["exc_key"]
    assert h["n_out"] == int((keys & 1 == 0).sum()) == int((codes == 0).sum()) > 0
    pos_to_idx = _padded_to_rowmajor(x.shape, (8, 8, 8))
    patched[pos_to_idx[(keys[keys & 1 == 1] >> 1).astype(np.int64)]] = True
    yy, ee = y.ravel(), expect.ravel()
    assert np.array_equal(yy[~patched].view(np.uint32), ee[~patched].view(np.uint32))


def _padded_to_rowmajor(shape, block):
    """Map padded block-major position -> row-major index (-1 if padding)."""
    shape3 = (1,) * (3 - len(shape)) + tuple(shape)
    block3 = (1,) * (3 - len(block)) + tuple(block)
    nb = [-(-n // b) for n, b in zip(shape3, block3)]
    z, y, x = np.meshgrid(*[np.arange(n) for n in shape3], indexing="ij")
    B = (z // block3[0] * nb[1] + y // block3[1]) * nb[2] + x // block3[2]
    inb = ((z % block3[0]) * block3[1] + y % block3[1]) * block3[2] + x % block3[2]
    pos = (B * (block3[0] * block3[1] * block3[2]) + inb).ravel()
    m = np.full(nb[0] * nb[1] * nb[2] * block3[0] * block3[1] * block3[2], -1, np.int64)
    m[pos] = np.arange(pos.size)
    return m


# --------------------------------------------------------------------------
# End to end: error bound, PSNR closed form, patches, degenerate inputs
# --------------------------------------------------------------------------

def _check_bound(x, y, eb_abs):
    xf = x.astype(np.float64).ravel()
    yf = y.astype(np.float64).ravel()
    fin = np.isfinite(xf)
    assert np.all(np.abs(xf[fin] - yf[fin]) <= eb_abs)
    # non-finite inputs come back bit-exact (stored verbatim)
    assert np.array_equal(x.ravel()[~fin].view(np.uint32), y.ravel()[~fin].view(np.uint32))


@pytest.mark.parametrize("valrel,expect_db", [(1e-3, 64.771), (1e-4, 84.771)])
def test_psnr_closed_form(orc, valrel, expect_db):
    """Dual-quant error is the prequantization rounding error, uniform on
    [-eb, eb] for a rough field, so RMSE = eb / sqrt(3) and PSNR =
    20 log10(sqrt(3) / valrel)."""
    from synth import fields
    x = fields.hurricane3d((40, 96, 96), seed=21)
    arc = orc.compress(x, valrel)
    y = orc.decompress(arc)
    eb_abs = au.header(arc)["eb_abs"]
    _check_bound(x, y, eb_abs)
    rng_ = float(x.max()) - float(x.min())
    rmse = math.sqrt(np.mean((x.astype(np.float64) - y) ** 2))
    psnr = 20 * math.log10(rng_ / rmse)
    assert abs(psnr - 20 * math.log10(math.sqrt(3) / valrel)) < 0.05
    assert abs(psnr - expect_db) < 0.05


def test_patches_keep_bound_at_large_magnitude(orc):
    """2^20 consecutive fp32 values far from zero: fp32 rounding of x * r and
    d° * h alone would overshoot eb; the rehearsal keeps every element
    within eb (Algorithm 1's watchdog idea)."""
    base = np.float32(3000.0)
    x = (base.view(np.uint32) + np.arange(1 << 20, dtype=np.uint32)).view(np.float32)
    # a power-of-two bound makes every product exact: no patch is needed
    assert au.header(orc.compress(x, 1.0 / 4096.0, mode=orc.EB_ABS))["n_patch"] == 0
    eb = 3.3e-4
    arc = orc.compress(x, eb, mode=orc.EB_ABS)
    y = orc.decompress(arc)
    _check_bound(x, y, eb)
    h = au.header(arc)
    assert h["n_patch"] > 0
    # without patches the plain dequantized values overshoot for some elements
    dq = orc.prequant(x, np.array([h["r_bits"]], np.uint32).view(np.float32)[0])
    plain = dq.astype(np.float32) * np.array([h["h_bits"]], np.uint32).view(np.float32)[0]
    assert np.sum(np.abs(plain.astype(np.float64) - x) > eb) == h["n_patch"]


@pytest.mark.parametrize("case", ["constant", "single", "empty", "all_outliers", "specials", "ragged1d",
                                  "tiny2d", "line3d", "radius1"])
def test_degenerate_inputs_round_trip(orc, case):
    rng = np.random.default_rng(42)
    kw = {}
    if case == "constant":
        x = np.full((9, 10, 11), 3.25, np.float32)
    elif case == "single":
        x = np.array([1.5], np.float32)
    elif case == "empty":
        x = np.zeros((0,), np.float32)
    elif case == "all_outliers":
        x = (rng.standard_normal((40, 40)) * 1e3).astype(np.float32)
        kw["mode"] = orc.EB_ABS   # eb 1e-4 absolute: every delta is far outside the cap
    elif case == "specials":
        x = rng.standard_normal(300).astype(np.float32)
        x[[3, 50, 51, 200]] = [np.nan, np.inf, -np.inf, -0.0]
        x[100] = np.float32(1e-40)
    elif case == "ragged1d":
        x = rng.standard_normal(33 * 32 + 5).astype(np.float32).cumsum()
    elif case == "tiny2d":
        x = rng.standard_normal((1, 3)).astype(np.float32)
    elif case == "line3d":
        x = rng.standard_normal((1, 1, 77)).astype(np.float32)
    elif case == "radius1":
        x = rng.standard_normal((5, 6, 7)).astype(np.float32)
        kw["radius"] = 1
    arc = orc.compress(x, 1e-4, **kw)
    y = orc.decompress(arc)
    assert y.shape == x.shape
    h = au.header(arc)
    _check_bound(x, y, h["eb_abs"])
    if case == "constant":
        assert h["eb_abs"] == 1e-4 and h["n_out"] == 8 and h["max_len"] == 1  # one outlier per block corner
    if case == "all_outliers":
        assert h["n_out"] > 0.9 * x.size
    if case == "radius1":
        assert h["n_out"] > 0 and h["radius"] == 1


def test_corrupt_archives_rejected(orc):
    from synth import fields
    x = fields.fourier2d((40, 50), seed=2)
    arc = orc.compress(x, 1e-4)
    bad = arc.copy()
    bad[0] ^= 1
    with pytest.raises(orc.OracleError) as e:
        orc.decompress(bad)
    assert e.value.status == orc.ECORRUPT
    with pytest.raises(orc.OracleError):
        orc.decompress(arc[:-4])
    bad = arc.copy()
    off = au.sections(arc)["offsets"]["len"]
    bad[off + 512] ^= 0x3  # damage the central code length -> Kraft sum != 1
    with pytest.raises(orc.OracleError):
        orc.decompress(bad)
    bad = arc.copy()
    off = au.sections(arc)["offsets"]["sub"]
    bad[off] ^= 1  # subchunk table disagrees with the stream
    with pytest.raises(orc.OracleError):
        orc.decompress(bad)


def test_archive_deterministic(orc):
    from synth import fields
    x = fields.hurricane3d((16, 24, 24), seed=3)
    assert np.array_equal(orc.compress(x, 1e-4), orc.compress(x, 1e-4))
