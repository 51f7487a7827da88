"""The entry point that allocates nothing (dqz_compress_async_static): its
workspace is the library's fixed per-GPU array.  Two calls in a row, the
second on a smaller field, each checked byte for byte against
dqz_compress_async on a context (and the result block against its result
block); a field whose workspace exceeds the fixed array is refused on the
host."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _result(dqz, buf):
    return dqz.dqz_result.from_buffer_copy(buf.cpu().numpy().tobytes())


def _pair(dqz, ctx, x, eb, mode):
    import torch
    t = torch.from_numpy(x).cuda()
    params = dqz.make_params(eb, mode)
    bound, ws = dqz.dqz_compress_bound(tuple(x.shape), params)
    ctx.dqz_ctx_reserve(ws)
    arcs, results = [], []
    for static in (True, False):
        arc = torch.full((bound,), 0xA5, dtype=torch.uint8, device="cuda")
        res = torch.zeros(dqz.DQZ_RESULT_BYTES, dtype=torch.uint8, device="cuda")
        if static:
            st = dqz.dqz_compress_async_static(t.data_ptr(), tuple(x.shape), params, arc.data_ptr(), bound,
                                               res.data_ptr())
        else:
            st = ctx.dqz_compress_async(t.data_ptr(), tuple(x.shape), params, arc.data_ptr(), bound, res.data_ptr())
        assert st == dqz.DQZ_OK
        torch.cuda.synchronize()
        r = _result(dqz, res)
        assert r.status == dqz.DQZ_OK, (static, r.status)
        arcs.append(arc[:r.archive_bytes].cpu().numpy())
        results.append(r)
    assert results[0].archive_bytes == results[1].archive_bytes
    assert bytes(results[0].header) == bytes(results[1].header)
    assert np.array_equal(arcs[0], arcs[1])
    return arcs[0]


def test_static_workspace_matches_context_path():
    import oracle
    from paper_2007_09625_amd import dqz
    from synth import fields
    ctx = dqz.Context(0)
    big = fields.hurricane3d((48, 96, 120), seed=61)
    small = fields.fourier2d((70, 130), seed=62)
    a = _pair(dqz, ctx, big, 1e-4, dqz.DQZ_EB_VALREL)
    b = _pair(dqz, ctx, small, 1e-3, dqz.DQZ_EB_VALREL)
    assert np.array_equal(a, oracle.compress(big, 1e-4))
    assert np.array_equal(b, oracle.compress(small, 1e-3))
    # absolute mode, and the larger field again after the smaller one
    c = _pair(dqz, ctx, big, 1e-2, dqz.DQZ_EB_ABS)
    assert np.array_equal(c, oracle.compress(big, 1e-2, oracle.EB_ABS))


def test_static_workspace_refuses_oversized_field():
    import torch
    from paper_2007_09625_amd import dqz
    shape = (400, 400, 400)          # workspace far above the fixed array
    params = dqz.make_params(1e-4)
    res = torch.zeros(dqz.DQZ_RESULT_BYTES, dtype=torch.uint8, device="cuda")
    x = torch.zeros(8, dtype=torch.float32, device="cuda")       # never read: refused on the host
    arc = torch.zeros(8, dtype=torch.uint8, device="cuda")
    st = dqz.dqz_compress_async_static(x.data_ptr(), shape, params, arc.data_ptr(), 1 << 40, res.data_ptr())
    assert st == dqz.DQZ_EUNSUPPORTED
