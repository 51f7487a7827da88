"""The host path: fields in host memory compressed slab by slab into a
container (copies overlapped with the kernels) and decompressed back.  The
container must be byte for byte the one built from the oracle's archives of
the same slabs; the decompressed field must be bit for bit the whole-field
decompression with the same absolute bound (prediction blocks never straddle
slabs), and within the bound on every element."""
from __future__ import annotations

import numpy as np
import pytest

import archive_util as au

pytestmark = pytest.mark.gpu


CASES = [
    ("3d", (37, 40, 52), 8 * 40 * 52 * 4 * 2, 1, 1e-4),      # 16-plane slabs, ragged last slab
    ("3d_abs", (20, 33, 47), 8 * 33 * 47 * 4, 0, 0.02),      # 8-plane slabs
    ("2d", (300, 410), 16 * 410 * 4 * 3, 1, 1e-3),           # 48-row slabs
    ("1d", (100003,), 32 * 4 * 400, 1, 1e-4),                 # 12,800-element slabs
    ("one_slab", (24, 40, 52), 1 << 30, 0, 0.01),
]


@pytest.mark.parametrize("name,shape,slab_bytes,mode,eb", CASES, ids=[c[0] for c in CASES])
def test_stream_container_matches_oracle_and_whole_field(name, shape, slab_bytes, mode, eb):
    import torch
    import oracle
    from paper_2007_09625_amd import dqz
    from synth import fields
    if len(shape) == 3:
        x = fields.hurricane3d(shape, seed=len(name))
    elif len(shape) == 2:
        x = fields.fourier2d(shape, seed=len(name))
    else:
        x = fields.particles1d(shape[0], seed=len(name), shuffle_block=512)
    ctx = dqz.Context(0)
    c = ctx.stream_compress(x, eb, mode, slab_bytes=slab_bytes)
    ref, arcs, eb_abs, rows = au.container_from_oracle(x, eb, mode, slab_bytes)
    assert c.size == ref.size and np.array_equal(c, ref)
    assert dqz.dqz_stream_info(c)[1:3] == (len(arcs), eb_abs)
    y = ctx.stream_decompress(c)
    # the whole field compressed with the same absolute bound decompresses identically
    t = torch.from_numpy(x).cuda()
    whole = ctx.decompress(ctx.compress(t, eb_abs, "abs")).cpu().numpy()
    assert np.array_equal(y.view(np.uint32), whole.view(np.uint32))
    # and equals the oracle's slab decompressions, concatenated
    ref_y = np.concatenate([oracle.decompress(a) for a in arcs], axis=0)
    assert np.array_equal(y.view(np.uint32), ref_y.view(np.uint32))
    xf, yf = x.astype(np.float64).ravel(), y.astype(np.float64).ravel()
    assert np.all(np.abs(xf - yf) <= eb_abs)
    if name == "one_slab":
        # one slab in absolute mode: the archive is the single-field archive
        assert np.array_equal(arcs[0], ctx.compress(t, eb, "abs").archive.cpu().numpy())


def test_stream_pinned_buffers_and_capacity():
    """Pinned host tensors as field, container and output; a container
    capacity below what the slabs need is DQZ_ETOOSMALL and the context
    stays usable."""
    import torch
    from paper_2007_09625_amd import dqz
    from synth import fields
    x = fields.hurricane3d((64, 48, 40), seed=9)
    xp = torch.from_numpy(x).pin_memory()
    ctx = dqz.Context(0)
    slab = 16 * 48 * 40 * 4
    ref, _, _, _ = au.container_from_oracle(x, 1e-3, 1, slab)
    cbuf = torch.empty(ref.size + 4096, dtype=torch.uint8).pin_memory()
    c = ctx.stream_compress(xp, 1e-3, "valrel", slab_bytes=slab, out=cbuf)
    assert np.array_equal(c.numpy(), ref)
    out = torch.empty(x.shape, dtype=torch.float32).pin_memory()
    y = ctx.stream_decompress(c, out=out)
    whole = ctx.decompress(ctx.compress(torch.from_numpy(x).cuda(), dqz.dqz_stream_info(ref)[2], "abs"))
    assert torch.equal(y.view(torch.int32), whole.cpu().view(torch.int32))
    small = torch.empty(ref.size // 2, dtype=torch.uint8).pin_memory()
    with pytest.raises(dqz.DqzError) as e:
        ctx.stream_compress(xp, 1e-3, "valrel", slab_bytes=slab, out=small)
    assert e.value.status == dqz.DQZ_ETOOSMALL
    c2 = ctx.stream_compress(x, 1e-3, "valrel", slab_bytes=slab)
    assert np.array_equal(c2, ref)


def test_stream_empty_field_and_damage():
    from paper_2007_09625_amd import dqz
    ctx = dqz.Context(0)
    x = np.zeros((0, 5), np.float32)
    c = ctx.stream_compress(x, 1e-3, "abs", slab_bytes=4096)
    assert dqz.dqz_stream_info(c)[:2] == ((0, 5), 0)
    assert ctx.stream_decompress(c).shape == (0, 5)
    from synth import fields
    y = fields.fourier2d((64, 64), seed=1)
    c = ctx.stream_compress(y, 1e-3, slab_bytes=16 * 64 * 4)
    bad = c.copy()
    offs = np.frombuffer(c[128:128 + 8 * 5].tobytes(), np.uint64)      # 4 slabs + end
    last = int(offs[3])
    sub = au.sections(c[last:int(offs[4])])["offsets"]["sub"]
    bad[last + sub] ^= 1      # the last slab's subchunk table disagrees with its stream
    with pytest.raises(dqz.DqzError) as e:
        ctx.stream_decompress(bad)
    assert e.value.status == dqz.DQZ_ECORRUPT
    assert np.array_equal(ctx.stream_decompress(c).view(np.uint32),
                          ctx.stream_decompress(c.copy()).view(np.uint32))
