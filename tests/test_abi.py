"""Host-side checks of libdqz: it loads, exports every declared entry point,
and its host-only functions (size bound, header parsing) agree with the
archives the oracle writes.  No GPU needed."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dqz.h")


@pytest.fixture(scope="module")
def dqz():
    from paper_2007_09625_amd import dqz as m
    return m


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dqz_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_names(dqz):
    assert declared_functions() == sorted(dqz.EXPORTED)


def test_library_exports_every_declared_symbol(dqz):
    out = subprocess.run(["nm", "-D", "--defined-only", dqz.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(\w+)", out))
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(dqz.lib, name)


def test_library_links_no_oracle(dqz):
    out = subprocess.run(["nm", "-D", dqz.LIB_PATH], capture_output=True, text=True, check=True).stdout
    assert "orc_" not in out
    ldd = subprocess.run(["ldd", dqz.LIB_PATH], capture_output=True, text=True).stdout
    assert "oracle" not in ldd


def test_status_strings(dqz):
    for st in range(0, -8, -1):
        assert dqz.lib.dqz_status_str(st)


def test_ctx_create_without_gpu_fails_cleanly(dqz):
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    h = ctypes.c_void_p()
    assert dqz.lib.dqz_ctx_create(0, 1 << 20, ctypes.byref(h)) == dqz.DQZ_EHIP
    assert not h.value


@pytest.mark.parametrize("shape", [(1000,), (37, 53), (9, 17, 33), (100, 500, 500), (0,), (1,)])
def test_compress_bound_covers_oracle_archives(dqz, orc, shape):
    rng = np.random.default_rng(0)
    n = int(np.prod(shape))
    if n > 100000:
        pytest.skip("large shape: bound arithmetic only")
    x = (rng.standard_normal(shape) * 100).astype(np.float32)
    for eb, mode in ((1e-4, 1), (1e-7, 0)):
        arc = orc.compress(x, eb, mode)
        bound, ws = dqz.dqz_compress_bound(shape, dqz.make_params(eb, mode))
        assert arc.size <= bound
        assert ws > 0


def test_compress_bound_rejects_bad_arguments(dqz):
    for shape in [(), (1, 2, 3, 4)]:
        with pytest.raises(dqz.DqzError):
            dqz.dqz_compress_bound(shape, dqz.make_params(1e-4))
    for kw in [dict(radius=3), dict(radius=8192), dict(sub_size=16), dict(sub_size=48), dict(chunk_subs=3)]:
        with pytest.raises(dqz.DqzError):
            dqz.dqz_compress_bound((100,), dqz.make_params(1e-4, **kw))
    with pytest.raises(dqz.DqzError) as e:
        dqz.dqz_compress_bound((1 << 31,), dqz.make_params(1e-4))
    assert e.value.status == dqz.DQZ_EUNSUPPORTED


@pytest.mark.parametrize("shape,eb,mode", [((300,), 1e-3, 1), ((40, 70), 1e-4, 1), ((10, 20, 30), 1e-2, 0)])
def test_archive_info_parses_oracle_headers(dqz, orc, shape, eb, mode):
    rng = np.random.default_rng(1)
    x = rng.standard_normal(shape).astype(np.float32).cumsum(-1)
    arc = orc.compress(x, eb, mode)
    got_shape, params, n, nbytes = dqz.dqz_archive_info(arc[:128].tobytes())
    assert got_shape == shape and n == x.size and nbytes == arc.size
    assert params.eb == eb and params.eb_mode == mode and params.radius == 512


def test_archive_info_rejects_damaged_headers(dqz, orc):
    x = np.random.default_rng(2).standard_normal((20, 30)).astype(np.float32)
    hdr = orc.compress(x, 1e-3)[:128].copy()
    for off in (0, 4, 6, 8, 44, 80, 96, 112, 120):
        bad = hdr.copy()
        bad[off] ^= 0x5A
        with pytest.raises(dqz.DqzError) as e:
            dqz.dqz_archive_info(bad.tobytes())
        assert e.value.status == dqz.DQZ_ECORRUPT
    with pytest.raises(dqz.DqzError):
        dqz.dqz_archive_info(hdr[:100].tobytes())


def test_package_has_no_cpu_fallback():
    import paper_2007_09625_amd.dqz as m
    src = open(m.__file__).read()
    assert "import oracle" not in src and "from oracle" not in src
    assert "numpy" not in src.split("def dqz_debug_copy")[0]


def test_workspace_bounds(dqz, orc):
    """The compress workspace bound covers the worst case (every element an
    outlier and a patch); the decompress bound parses the header and grows
    with the field; both reject bad input."""
    small = dqz.dqz_compress_bound((1000,), dqz.make_params(1e-4))[1]
    big = dqz.dqz_compress_bound((100, 500, 500), dqz.make_params(1e-4))[1]
    assert big > 16 * 25_000_000 > small > 16 * 1000
    x = np.random.default_rng(4).standard_normal((20, 30, 40)).astype(np.float32)
    arc = orc.compress(x, 1e-4)
    ws = dqz.dqz_decompress_bound(arc[:128].tobytes())
    assert ws >= 2 * x.size
    empty = orc.compress(np.zeros(0, np.float32), 1e-4)
    assert dqz.dqz_decompress_bound(empty[:128].tobytes()) == 0
    bad = arc[:128].copy()
    bad[0] ^= 1
    with pytest.raises(dqz.DqzError) as e:
        dqz.dqz_decompress_bound(bad.tobytes())
    assert e.value.status == dqz.DQZ_ECORRUPT


def test_result_struct_layout(dqz):
    """dqz_result as declared in include/dqz.h: status at byte 4, sizes at 8 and
    16, the header at 32 (the library checks the same layout at compile time)."""
    r = dqz.dqz_result
    assert r.status.offset == 4 and r.archive_bytes.offset == 8 and r.workspace_need.offset == 16
    assert r.header.offset == 32 and dqz.DQZ_RESULT_BYTES == 160


def test_null_context_arguments(dqz):
    """Entry points reject a NULL context without touching the GPU."""
    assert dqz.lib.dqz_ctx_reserve(None, 100) == dqz.DQZ_EINVAL
    assert dqz.lib.dqz_ctx_workspace(None, None, None) == dqz.DQZ_EINVAL
    assert dqz.lib.dqz_debug_inject(None, dqz.DQZ_INJECT_ALLOC_FAIL, 1) == dqz.DQZ_EINVAL
    s = dqz.make_shape((100,))
    p = dqz.make_params(1e-4)
    assert dqz.lib.dqz_compress_async(None, None, ctypes.byref(s), ctypes.byref(p), None, 0, None, None) == dqz.DQZ_EINVAL
    assert dqz.lib.dqz_decompress_async(None, None, 0, None, None, 0, None, None) == dqz.DQZ_EINVAL


def test_stream_info_parses_containers_and_rejects_damage(dqz, orc):
    """dqz_stream_info (host only) on containers built from the oracle's slab
    archives: shape, slab count and absolute bound; damaged headers, offsets
    and slab shapes are rejected."""
    import archive_util as au
    from synth import fields
    x = fields.hurricane3d((37, 20, 30), seed=3)
    c, arcs, eb_abs, rows = au.container_from_oracle(x, 1e-3, 1, slab_bytes=16 * 20 * 30 * 4)
    assert rows == 16 and len(arcs) == 3
    shape, n, eb, ws = dqz.dqz_stream_info(c)
    assert shape == x.shape and n == 3 and eb == eb_abs and ws > 0
    for off, val in ((0, 0x00), (6, 4), (32, 3), (40, 9), (80, 1)):
        bad = c.copy()
        bad[off] ^= val if val else 0xFF
        with pytest.raises(dqz.DqzError) as e:
            dqz.dqz_stream_info(bad)
        assert e.value.status == dqz.DQZ_ECORRUPT
    bad = c.copy()
    bad[128 + 8] ^= 8                       # slab 1 starts elsewhere
    with pytest.raises(dqz.DqzError):
        dqz.dqz_stream_info(bad)
    bad = c.copy()
    o1 = int(np.frombuffer(c[136:144].tobytes(), np.uint64)[0])
    bad[o1 + 8] ^= 1                        # slab 1's archive claims another extent
    with pytest.raises(dqz.DqzError):
        dqz.dqz_stream_info(bad)
    with pytest.raises(dqz.DqzError):
        dqz.dqz_stream_info(c[:-1])
