"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bar: archive bytes bit-exact (codes, histogram-derived lengths, exception
lists, tables and bitstream are all inside the archive), decompressed floats
bit-exact, and |x - x'| <= eb_abs on every element.
"""
from __future__ import annotations

import numpy as np
import pytest

import archive_util as au

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2007_09625_amd import dqz
    return dqz.Context(0)


def _gpu_round_trip(ctx, x, eb, mode, **kw):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    comp = ctx.compress(t, eb, mode, **kw)
    y = ctx.decompress(comp)
    torch.cuda.synchronize()
    return comp.archive.cpu().numpy(), comp.header, y.cpu().numpy()


def _explain_mismatch(ctx, x, eb, mode, gpu_arc, ref_arc, **kw):
    """Locate the first differing stage for the failure message."""
    import torch
    from paper_2007_09625_amd import dqz
    lines = []
    # the stage dumps hold the most recent compression: compress again (the
    # round trip's decompression has overwritten them)
    ctx.compress(torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0"), eb, mode, **kw)
    torch.cuda.synchronize()
    if gpu_arc.size != ref_arc.size:
        lines.append(f"archive sizes differ: gpu {gpu_arc.size} oracle {ref_arc.size}")
    else:
        d = np.nonzero(gpu_arc != ref_arc)[0]
        lines.append(f"{d.size} bytes differ, first at {d[:8].tolist()}")
    try:
        gs, rs = au.sections(gpu_arc), au.sections(ref_arc)
        lines.append(f"section offsets {rs['offsets']}")
        for k in ("lengths", "chunks", "subs", "exc_key", "exc_payload", "stream"):
            a, b = gs[k], rs[k]
            if a.shape != b.shape or not np.array_equal(a, b):
                idx = int(np.argmax(a[:min(a.size, b.size)] != b[:min(a.size, b.size)])) if min(a.size, b.size) else 0
                lines.append(f"section {k} differs: sizes {a.size} vs {b.size}, first diff at {idx}")
        gh, rh = gs["header"], rs["header"]
        for k in gh:
            if gh[k] != rh[k]:
                lines.append(f"header {k}: gpu {gh[k]} oracle {rh[k]}")
        import oracle
        _, codes, freq, _ = oracle.stages(x, eb, mode, gh["radius"])
        hist = ctx.dqz_debug_copy(dqz.DQZ_DBG_HISTOGRAM, 4 * 2 * gh["radius"]).view(np.uint32)
        if not np.array_equal(hist.astype(np.uint64), freq):
            lines.append(f"histogram differs at bins {np.nonzero(hist != freq)[0][:10]}")
        padded = gs["padded"]
        gcodes = ctx.dqz_debug_copy(dqz.DQZ_DBG_CODES, 2 * padded).view(np.uint16)
        real = gcodes[gcodes != 0xFFFF]
        if real.size != codes.size or not np.array_equal(real, codes):
            d = np.nonzero(real[:codes.size] != codes[:real.size])[0]
            lines.append(f"codes differ: {real.size} vs {codes.size} real codes, first diffs {d[:10]}")
    except Exception as e:  # pragma: no cover - diagnostics only
        lines.append(f"(diagnostics failed: {e!r})")
    return "\n".join(lines)


def _check(ctx, x, eb=1e-4, mode=1, **kw):
    import oracle
    gpu_arc, hdr, y = _gpu_round_trip(ctx, x, eb, mode, **kw)
    okw = {k: v for k, v in kw.items()}
    ref_arc = oracle.compress(x, eb, mode, **{"radius": okw.get("radius", 512),
                                               "sub_size": okw.get("sub_size", 128),
                                               "chunk_subs": okw.get("chunk_subs", 64),
                                               "layers": okw.get("layers", 1) or 1})
    if not np.array_equal(gpu_arc, ref_arc):
        pytest.fail("archive differs from the oracle\n" + _explain_mismatch(ctx, x, eb, mode, gpu_arc, ref_arc, **kw))
    assert hdr == ref_arc[:128].tobytes()
    ref_y = oracle.decompress(ref_arc)
    assert y.shape == x.shape
    assert np.array_equal(y.view(np.uint32), ref_y.view(np.uint32)), "decompressed floats differ from the oracle"
    eb_abs = au.header(ref_arc)["eb_abs"]
    xf, yf = x.astype(np.float64).ravel(), y.astype(np.float64).ravel()
    fin = np.isfinite(xf)
    assert np.all(np.abs(xf[fin] - yf[fin]) <= eb_abs)
    return ref_arc


SHAPES_3D = [(8, 8, 8), (9, 17, 70), (24, 40, 52), (1, 1, 77), (3, 70, 5), (16, 16, 520), (33, 65, 130)]
SHAPES_2D = [(1, 3), (16, 16), (45, 70), (17, 300), (200, 600), (3, 4100)]
SHAPES_1D = [(1,), (33,), (4096,), (4097,), (100003,), ((1 << 20) + 3,)]


@pytest.mark.parametrize("shape", SHAPES_3D + SHAPES_2D + SHAPES_1D, ids=str)
def test_parity_shapes(ctx, shape):
    from synth import fields
    if len(shape) == 3:
        x = fields.hurricane3d(shape, seed=sum(shape))
    elif len(shape) == 2:
        x = fields.fourier2d(shape, seed=sum(shape))
    else:
        x = fields.particles1d(shape[0], seed=shape[0] % 97, shuffle_block=512)
    _check(ctx, x)


@pytest.mark.parametrize("eb,mode", [(1e-2, 1), (1e-3, 1), (1e-5, 1), (1e-3, 0), (0.25, 0)])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_parity_error_bounds(ctx, eb, mode, ndim):
    from synth import fields
    x = {1: lambda: fields.particles1d(50000, seed=5, shuffle_block=256),
         2: lambda: fields.fourier2d((70, 90), seed=6),
         3: lambda: fields.hurricane3d((20, 30, 40), seed=7)}[ndim]()
    _check(ctx, x, eb, mode)


@pytest.mark.parametrize("sub_size,chunk_subs", [(32, 1), (64, 4), (128, 64), (256, 128), (512, 2), (1024, 65536)])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_parity_table_geometry(ctx, sub_size, chunk_subs, ndim):
    from synth import fields
    x = {1: lambda: fields.particles1d(70001, seed=8, shuffle_block=128),
         2: lambda: fields.fourier2d((100, 130), seed=9),
         3: lambda: fields.hurricane3d((17, 45, 70), seed=10)}[ndim]()
    _check(ctx, x, 1e-4, 1, sub_size=sub_size, chunk_subs=chunk_subs)


@pytest.mark.parametrize("radius", [1, 2, 8, 64, 1024])
def test_parity_radius(ctx, radius):
    from synth import fields
    x = fields.hurricane3d((16, 24, 40), seed=radius)
    _check(ctx, x, 1e-4, 1, radius=radius)


@pytest.mark.parametrize("case", ["constant", "specials", "all_outliers", "large_magnitude", "zeros", "tiny_eb"])
def test_parity_degenerate(ctx, case):
    rng = np.random.default_rng(3)
    mode, eb = 1, 1e-4
    if case == "constant":
        x = np.full((10, 20, 30), -7.5, np.float32)
    elif case == "specials":
        x = rng.standard_normal((40, 50)).astype(np.float32)
        x.ravel()[[0, 7, 100, 999, 1500]] = [np.nan, np.inf, -np.inf, -0.0, 1e-42]
    elif case == "all_outliers":
        x = (rng.standard_normal(20000) * 1e4).astype(np.float32)
        mode, eb = 0, 1e-3
    elif case == "large_magnitude":
        base = np.float32(3000.0)
        x = (base.view(np.uint32) + np.arange(1 << 16, dtype=np.uint32)).view(np.float32).reshape(64, 1024)
        mode, eb = 0, 3.3e-4
    elif case == "zeros":
        x = np.zeros((5, 6, 7), np.float32)
    elif case == "tiny_eb":
        x = rng.standard_normal((30, 30, 30)).astype(np.float32)
        eb = 1e-7
    _check(ctx, x, eb, mode)


def test_parity_empty_field(ctx):
    import torch
    import oracle
    x = np.zeros((0,), np.float32)
    t = torch.zeros((0,), dtype=torch.float32, device="cuda:0")
    comp = ctx.compress(t, 1e-4)
    assert np.array_equal(comp.archive.cpu().numpy(), oracle.compress(x, 1e-4))
    y = ctx.decompress(comp)
    assert y.numel() == 0


def test_archive_deterministic_and_reusable_context(ctx):
    import torch
    from synth import fields
    x = torch.from_numpy(fields.hurricane3d((30, 64, 64), seed=1)).cuda()
    a = ctx.compress(x, 1e-4).archive.cpu().numpy()
    small = torch.from_numpy(fields.fourier2d((20, 20), seed=2)).cuda()
    ctx.compress(small, 1e-3)
    b = ctx.compress(x, 1e-4).archive.cpu().numpy()
    assert np.array_equal(a, b)


def test_gpu_decodes_oracle_archive_and_rejects_damage(ctx):
    """The decoder accepts the oracle's archive and reports damaged tables."""
    import torch
    import oracle
    from paper_2007_09625_amd import dqz
    from synth import fields
    x = fields.hurricane3d((20, 30, 40), seed=4)
    arc = oracle.compress(x, 1e-4)
    y = ctx.decompress(torch.from_numpy(arc).cuda())
    assert np.array_equal(y.cpu().numpy().view(np.uint32), oracle.decompress(arc).view(np.uint32))
    bad = arc.copy()
    bad[au.sections(arc)["offsets"]["sub"]] ^= 1      # subchunk table disagrees with the stream
    with pytest.raises(dqz.DqzError) as e:
        ctx.decompress(torch.from_numpy(bad).cuda())
    assert e.value.status == dqz.DQZ_ECORRUPT
    bad = arc.copy()
    bad[au.sections(arc)["offsets"]["len"] + 512] ^= 3   # lengths no longer a complete prefix code
    with pytest.raises(dqz.DqzError) as e:
        ctx.decompress(torch.from_numpy(bad).cuda())
    assert e.value.status == dqz.DQZ_ECORRUPT


def test_capacity_too_small(ctx):
    import torch
    from paper_2007_09625_amd import dqz
    from synth import fields
    x = torch.from_numpy(fields.hurricane3d((16, 32, 32), seed=5)).cuda()
    good = ctx.compress(x, 1e-4)
    out = torch.empty(good.nbytes - 1, dtype=torch.uint8, device="cuda:0")
    st, need, _ = ctx.dqz_compress(x.data_ptr(), tuple(x.shape), dqz.make_params(1e-4), out.data_ptr(), out.numel())
    assert st == dqz.DQZ_ETOOSMALL and need == good.nbytes
    st, need, _ = ctx.dqz_compress(x.data_ptr(), tuple(x.shape), dqz.make_params(1e-4), out.data_ptr(), 100)
    assert st == dqz.DQZ_ETOOSMALL


@pytest.mark.parametrize("name,eb", [("c1", 1e-4), ("c2", 1e-4), ("c2", 1e-3)])
def test_parity_full_size_workloads(ctx, name, eb):
    """The 2D 1800x3600 and 3D 100x500x500 workloads at full size, in the
    launch configuration the benchmark times."""
    from synth import fields
    x = fields.workload(name)
    arc = _check(ctx, x, eb, 1)
    h = au.header(arc)
    print(f"{name} eb={eb}: {x.nbytes / arc.size:.2f}x, {8 * arc.size / x.size:.3f} bits/elem, "
          f"outliers {h['n_out']}, patches {h['n_patch']}, max_len {h['max_len']}")


def _fibonacci_field(k, seed):
    """1D field (absolute eb 0.5, so prequant is the identity on integers) whose
    Lorenzo deltas take k values with Fibonacci frequencies: the Huffman tree is
    a chain and the longest code has k - 1 bits.  Values are rebuilt from the
    chosen deltas block by block (1D blocks of 32), so every delta is exact."""
    fib = [1, 1]
    while len(fib) < k:
        fib.append(fib[-1] + fib[-2])
    deltas = np.repeat(np.arange(-(k // 2), k - k // 2, dtype=np.int64), fib[:k])
    rng = np.random.default_rng(seed)
    rng.shuffle(deltas)
    n = deltas.size
    pad = (-n) % 32
    blocks = np.concatenate([deltas, np.zeros(pad, np.int64)]).reshape(-1, 32)
    x = np.cumsum(blocks, axis=1).ravel()[:n]
    assert np.abs(x).max() < (1 << 24)
    return x.astype(np.float32)


@pytest.mark.parametrize("k", [28, 35], ids=["max_len27", "max_len34"])
def test_parity_long_codes(ctx, k):
    """Codes longer than 24 bits take the 64-bit codeword path of the encoder;
    codes longer than 32 bits take the decoder's window restart."""
    x = _fibonacci_field(k, seed=k)
    arc = _check(ctx, x, 0.5, 0, radius=64)
    assert au.header(arc)["max_len"] == k - 1


def test_parity_wide_sort_keys(ctx):
    """A symbol count of 2^21 or more with 2048 symbols (radius 1024) leaves no
    room for (count, symbol) in 32 bits: the codebook sorts its leaves on
    64-bit keys.  Sparse integer spikes on a zero field at absolute eb 0.5."""
    rng = np.random.default_rng(21)
    n = (1 << 21) + 300_000
    x = np.zeros(n, np.float32)
    idx = rng.choice(n, n // 100, replace=False)
    x[idx] = rng.integers(-400, 400, idx.size).astype(np.float32)
    arc = _check(ctx, x, 0.5, 0, radius=1024)
    import oracle
    _, _, freq, _ = oracle.stages(x, 0.5, 0, 1024)
    assert int(freq.max()) >= 1 << 21


def test_stage_timing_modes(ctx):
    """Timing level 1 reports every stage; DQZ_TIMING_STAGE(which, stage)
    reports the chosen stage only; the archive is the same either way."""
    import torch
    from paper_2007_09625_amd import dqz
    from synth import fields
    x = torch.from_numpy(fields.hurricane3d((24, 40, 52), seed=3)).cuda()
    ctx.dqz_ctx_set_timing(1)
    a1 = ctx.compress(x, 1e-4).archive.cpu().numpy()
    full = ctx.dqz_stage_times(0)
    assert list(full) == list(dqz.COMPRESS_STAGES)
    assert full["quantize"] > 0 and full["encode"] > 0
    ctx.dqz_ctx_set_timing(dqz.timing_stage(0, "encode"))
    a2 = ctx.compress(x, 1e-4).archive.cpu().numpy()
    one = ctx.dqz_stage_times(0)
    assert one["encode"] > 0 and all(v == 0 for k, v in one.items() if k != "encode")
    ctx.dqz_ctx_set_timing(0)
    assert np.array_equal(a1, a2)
    with pytest.raises(Exception):
        ctx.dqz_ctx_set_timing(0x100 | (2 << 4))
    # level 2: the decoding waves' phase sums, readable after the decompression
    ctx.dqz_ctx_set_timing(2)
    c = ctx.compress(x, 1e-4)
    y = ctx.decompress(c)
    ph = ctx.dqz_debug_copy(dqz.DQZ_DBG_PHASES, 256).view(np.uint64)
    ctx.dqz_ctx_set_timing(0)
    assert ph[24] <= ph[25] and ph[26] > 0 and ph[27] > 0
    assert np.array_equal(y.cpu().numpy().view(np.uint32), ctx.decompress(c).cpu().numpy().view(np.uint32))


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_parity_wraparound(ctx, ndim):
    """Absolute eb 0.5 (prequantization is the identity on integers) on values
    of magnitude near 1e9 with alternating signs: the mixed Lorenzo differences
    (up to 2^ndim * 1e9) wrap modulo 2^32, every delta is an outlier record
    with a wrapped payload, and the inverse prefix sums wrap back (Sec. 3.1.2;
    the forward and inverse maps are bijections modulo 2^32)."""
    rng = np.random.default_rng(40 + ndim)
    shape = {1: (5000,), 2: (37, 45), 3: (11, 13, 17)}[ndim]
    idx = np.indices(shape).sum(axis=0)
    sign = np.where(idx % 2 == 0, 1.0, -1.0)
    mag = 1e9 - 64.0 * rng.integers(0, 100, shape)      # multiples of 64: exact in fp32
    x = (sign * mag).astype(np.float32)
    x.ravel()[::7] = rng.integers(-300, 300, x.size)[::7].astype(np.float32)   # some in-cap codes
    arc = _check(ctx, x, 0.5, 0)
    assert au.header(arc)["n_out"] > x.size // 2


@pytest.fixture(scope="module")
def c3_field():
    from synth import fields
    return fields.workload("c3")


@pytest.mark.timeout(900)
@pytest.mark.parametrize("eb", [1e-4, 1e-3])
def test_parity_full_size_c3(ctx, c3_field, eb):
    """The 1D 280,953,867-element particle workload at full size (HACC shape,
    Sec. 4.1): whole archive bytes and decompressed float bits against the
    oracle, |x - x'| <= eb_abs on every element."""
    arc = _check(ctx, c3_field, eb, 1)
    h = au.header(arc)
    print(f"c3 eb={eb}: {c3_field.nbytes / arc.size:.2f}x, {8 * arc.size / c3_field.size:.3f} bits/elem, "
          f"outliers {h['n_out']}, patches {h['n_patch']}, max_len {h['max_len']}", flush=True)


# --------------------------------------------------------------------------
# The 2-layer Lorenzo predictor (the generalized predictor of Sec. 3.1.2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(8, 8, 8), (9, 17, 70), (33, 65, 130), (45, 70), (200, 600), (3, 4100),
                                   (33,), (100003,)], ids=str)
@pytest.mark.parametrize("eb", [1e-4, 1e-2])
def test_parity_two_layers(ctx, shape, eb):
    from synth import fields
    if len(shape) == 3:
        x = fields.hurricane3d(shape, seed=sum(shape))
    elif len(shape) == 2:
        x = fields.fourier2d(shape, seed=sum(shape))
    else:
        x = fields.particles1d(shape[0], seed=shape[0] % 97, shuffle_block=512)
    arc = _check(ctx, x, eb, 1, layers=2)
    assert int(arc[117]) == 1


@pytest.mark.parametrize("sub_size,chunk_subs", [(32, 1), (256, 128), (512, 2)])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_parity_two_layers_other_subchunks(ctx, sub_size, chunk_subs, ndim):
    """Subchunk sizes other than 128 decode in the one-kernel decoder."""
    from synth import fields
    x = {1: lambda: fields.particles1d(70001, seed=8, shuffle_block=128),
         2: lambda: fields.fourier2d((100, 130), seed=9),
         3: lambda: fields.hurricane3d((17, 45, 70), seed=10)}[ndim]()
    _check(ctx, x, 1e-4, 1, sub_size=sub_size, chunk_subs=chunk_subs, layers=2)


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_parity_two_layers_wraparound(ctx, ndim):
    rng = np.random.default_rng(50 + ndim)
    shape = {1: (5000,), 2: (37, 45), 3: (11, 13, 17)}[ndim]
    idx = np.indices(shape).sum(axis=0)
    x = (np.where(idx % 2 == 0, 1.0, -1.0) * (1e9 - 64.0 * rng.integers(0, 100, shape))).astype(np.float32)
    _check(ctx, x, 0.5, 0, layers=2)


def test_four_dimensional_field_flattened(ctx):
    """A 4D field (QMCPACK-like, Sec. 4.1's dataset table) is compressed as
    3D with its two slowest axes merged."""
    import torch
    import oracle
    from synth import fields
    x4 = fields.hurricane3d((12, 23, 23), seed=4).reshape(3, 4, 23, 23)
    t = torch.from_numpy(x4).cuda()
    c = ctx.compress(t, 1e-4)
    ref = oracle.compress(x4.reshape(12, 23, 23), 1e-4)
    assert np.array_equal(c.archive.cpu().numpy(), ref)
    y = ctx.decompress(c, out=torch.empty_like(t).view(12, 23, 23))
    assert np.array_equal(y.cpu().numpy().view(np.uint32), oracle.decompress(ref).view(np.uint32))


def test_parity_two_layers_full_size_3d(ctx):
    from synth import fields
    x = fields.workload("c2")
    arc = _check(ctx, x, 1e-4, 1, layers=2)
    h = au.header(arc)
    print(f"c2 2-layer eb=1e-4: {x.nbytes / arc.size:.3f}x, outliers {h['n_out']}, max_len {h['max_len']}")


@pytest.mark.parametrize("ndim", [1, 2])
def test_parity_record_density_per_unit(ctx, ndim):
    """Units of 512 positions with 0 to 35 spikes each (about two outliers
    per spike: from no records to well over 64 in one unit), and in every
    fifth unit a run of values near 3000 whose rounding makes patches:
    exercises both ways reconstruction takes a unit's exception records (a
    scalar walk for a few, the per-lane LDS scatter for more) and the
    boundary between them."""
    rng = np.random.default_rng(11 + ndim)
    n_units = 96
    x = (np.float32(3.0) + np.cumsum(rng.standard_normal(512 * n_units) * 1e-3)).astype(np.float32)
    for u in range(n_units):
        pos = 512 * u + rng.choice(512, size=u % 36, replace=False)
        x[pos] += np.float32(50.0)
        if u % 5 == 0:
            x[512 * u + 100:512 * u + 164] += np.float32(2997.0)
    if ndim == 2:
        x = x.reshape(96, 512)   # 16x16 blocks: a unit is two of them
    _check(ctx, x, 3.3e-4, 0)
