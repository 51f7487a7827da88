"""Archive section parser used by the tests (format layout only).

Header (128 bytes, little-endian) and section order:
  lengths u8[2R] @128, chunk offsets u64[n_chunks] @align8(128+2R),
  subchunk bits u16[n_sub], exceptions {u32 key, u32 payload}[n_out+n_patch]
  @align8, stream u32[ceil(total_bits/32)].
"""
from __future__ import annotations

import struct

import numpy as np

HEADER = struct.Struct("<IHBB3Q3IIddIIIIQIIQIIIB3xQ")
FIELDS = ("magic", "version", "ndim", "eb_mode", "nz", "ny", "nx", "bz", "by", "bx", "radius",
          "eb_param", "eb_abs", "h_bits", "r_bits", "vmin_bits", "vmax_bits", "n_elems", "n_out",
          "n_patch", "total_bits", "sub_size", "chunk_subs", "n_chunks", "max_len", "archive_bytes")
assert HEADER.size == 128


def header(arc) -> dict:
    b = np.asarray(arc, dtype=np.uint8)[:128].tobytes()
    return dict(zip(FIELDS, HEADER.unpack(b)))


def _a8(v):
    return (v + 7) // 8 * 8


def sections(arc) -> dict:
    arc = np.asarray(arc, dtype=np.uint8)
    h = header(arc)
    R = h["radius"]
    nb = [-(-h[a] // h[b]) for a, b in (("nz", "bz"), ("ny", "by"), ("nx", "bx"))]
    padded = nb[0] * nb[1] * nb[2] * h["bz"] * h["by"] * h["bx"]
    n_sub = -(-padded // h["sub_size"])
    n_chunks = -(-n_sub // h["chunk_subs"])
    off_len = 128
    off_chunk = _a8(off_len + 2 * R)
    off_sub = off_chunk + 8 * n_chunks
    off_exc = _a8(off_sub + 2 * n_sub)
    n_exc = h["n_out"] + h["n_patch"]
    off_str = off_exc + 8 * n_exc
    n_words = -(-h["total_bits"] // 32)
    end = off_str + 4 * n_words
    exc = arc[off_exc:off_str].view(np.uint32).reshape(-1, 2) if n_exc else np.zeros((0, 2), np.uint32)
    return dict(
        header=h,
        padded=padded,
        lengths=arc[off_len:off_len + 2 * R].copy(),
        chunks=arc[off_chunk:off_sub].view(np.uint64).copy(),
        subs=arc[off_sub:off_sub + 2 * n_sub].view(np.uint16).copy(),
        exc_key=exc[:, 0].copy(),
        exc_payload=exc[:, 1].copy(),
        stream=arc[off_str:end].view(np.uint32).copy() if n_words else np.zeros(0, np.uint32),
        end=end,
        offsets=dict(len=off_len, chunk=off_chunk, sub=off_sub, exc=off_exc, str=off_str),
    )


def stream_bits(words: np.ndarray, total_bits: int) -> np.ndarray:
    """Stream bit i = bit (31 - i mod 32) of word i // 32, as a 0/1 array."""
    w = np.asarray(words, dtype=np.uint32)
    bits = ((w[:, None] >> np.arange(31, -1, -1, dtype=np.uint32)[None, :]) & 1).astype(np.uint8)
    return bits.ravel()[:total_bits]


# -- streaming containers ('DQZS'): 128-byte header, (slabs + 1) u64 offsets,
#    slab archives each 8-byte aligned --------------------------------------
STREAM_MAGIC = 0x535A5144
BLOCK_EDGE = {1: 32, 2: 16, 3: 8}


def slab_rows(shape, slab_bytes):
    """Slab extent along the slowest axis for a slab size in bytes."""
    row = int(np.prod(shape[1:])) if len(shape) > 1 else 1
    e = BLOCK_EDGE[len(shape)]
    rows = slab_bytes // (4 * row) if row else shape[0]
    rows = rows // e * e
    return int(min(max(rows, e), shape[0]))


def container_from_oracle(x, eb, mode, slab_bytes, radius=512, sub_size=128, chunk_subs=64):
    """The container the streaming compression must write, built from the
    oracle's archives of each slab (absolute bound: eb, or eb times the whole
    field's finite range in the value-range-relative mode)."""
    import oracle
    x = np.ascontiguousarray(x, dtype=np.float32)
    shape = x.shape
    vmin, vmax, nfin = oracle.value_range(x)
    eb_abs = oracle.eb_params(mode, eb, vmin, vmax, nfin)[0]
    rows = slab_rows(shape, slab_bytes) if x.size else 0
    n_slabs = -(-shape[0] // rows) if x.size else 0
    arcs = [oracle.compress(x[k * rows:(k + 1) * rows], eb_abs, oracle.EB_ABS, radius=radius, sub_size=sub_size,
                            chunk_subs=chunk_subs) for k in range(n_slabs)]
    off = _a8(128 + 8 * (n_slabs + 1))
    offsets = []
    for a in arcs:
        offsets.append(off)
        off = _a8(off + a.size)
    total = offsets[-1] + arcs[-1].size if arcs else _a8(128 + 8)
    offsets.append(total)
    dims = [1] * (3 - len(shape)) + list(shape)
    h = bytearray(128)
    struct.pack_into("<IHBB3QQII", h, 0, STREAM_MAGIC, 1, len(shape), mode, *dims, rows, n_slabs, radius)
    struct.pack_into("<dd", h, 48, eb, eb_abs)
    if mode == 1 and nfin:
        struct.pack_into("<ff", h, 64, vmin, vmax)
    struct.pack_into("<QQII", h, 72, x.size, total, sub_size, chunk_subs)
    out = np.zeros(total, np.uint8)
    out[:128] = np.frombuffer(bytes(h), np.uint8)
    out[128:128 + 8 * len(offsets)] = np.frombuffer(np.array(offsets, np.uint64).tobytes(), np.uint8)
    for o, a in zip(offsets, arcs):
        out[o:o + a.size] = a
    return out, arcs, eb_abs, rows
