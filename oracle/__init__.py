"""CPU oracle of the cuSZ compression method (test infrastructure only).

This package wraps ``dqz_oracle.c`` -- a plain, single-threaded C
implementation of the paper's pipeline written for checking by eye -- via
ctypes.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product path never does.  It shares no code with
the HIP implementation.

Functions follow the paper's steps:
  value_range / eb_params   -- value-range-relative error bound (footnote, Sec. 3.2.2)
  prequant                  -- prequantization (Sec. 3.1.2, Algorithm 2)
  lorenzo_delta             -- 1- and 2-layer Lorenzo + zero padding layer (Sec. 3.1.1-3.1.2)
  lorenzo_reconstruct       -- cascading reconstruction (Algorithm 2, decompression)
  huffman_lengths           -- Huffman tree code lengths (Sec. 3.2.2)
  canonical_codes           -- canonical codebook (Sec. 3.2.3)
  compress / decompress     -- the whole pipeline (Sec. 3.1-3.3)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dqz_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "libdqz_oracle.so")

OK, EINVAL, ETOOSMALL, ENOMEM, ECORRUPT, EUNSUPPORTED = 0, -1, -2, -3, -4, -5

EB_ABS, EB_VALREL = 0, 1
HEADER_BYTES = 128


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


def build() -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    tmp = f"{_LIB_PATH}.{os.getpid()}.{threading.get_ident()}.tmp"
    cmd = ["gcc", "-O2", "-std=gnu99", "-Wall", "-ffp-contract=off", "-fno-fast-math",
           "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None
_lib_lock = threading.Lock()


def _load():
    global _lib
    if _lib is not None:
        return _lib
    with _lib_lock:   # callers on several host threads build and bind it once
        if _lib is None:
            _lib = _bind()
    return _lib


def _bind():
    path = os.environ.get("DQZ_ORACLE_LIB")   # a deliberately mutated build (mutation tests)
    if not path:
        path = _LIB_PATH
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build()
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    u64, i32, u32, f64 = ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32, ctypes.c_double
    lib.orc_value_range.argtypes = [P, u64, P, P, P]
    lib.orc_eb_params.argtypes = [i32, f64, ctypes.c_float, ctypes.c_float, u64, P, P, P]
    lib.orc_prequant.argtypes = [P, u64, ctypes.c_float, P]
    lib.orc_prequant.restype = None
    lib.orc_lorenzo_delta.argtypes = [P, i32, P, P]
    lib.orc_lorenzo_reconstruct.argtypes = [P, i32, P, P]
    lib.orc_huffman_lengths.argtypes = [P, u32, P]
    lib.orc_canonical_codes.argtypes = [P, u32, P]
    lib.orc_compress.argtypes = [P, i32, P, f64, i32, u32, u32, u32, P, u64, P]
    lib.orc_compress_layers.argtypes = [P, i32, P, f64, i32, u32, u32, u32, i32, P, u64, P]
    lib.orc_lorenzo_delta_n.argtypes = [P, i32, P, i32, P]
    lib.orc_lorenzo_reconstruct_n.argtypes = [P, i32, P, i32, P]
    lib.orc_compressed_size.argtypes = [P, i32, P, f64, i32, u32, u32, u32, P]
    lib.orc_decompress.argtypes = [P, u64, P, u64]
    lib.orc_stages.argtypes = [P, i32, P, f64, i32, u32, P, P, P, P]
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _dims(shape) -> np.ndarray:
    return np.ascontiguousarray(np.array(list(shape), dtype=np.uint64))


def value_range(x: np.ndarray):
    """Finite min / max under IEEE total order and the finite count."""
    x = np.ascontiguousarray(x, dtype=np.float32).ravel()
    lo = np.zeros(1, np.float32)
    hi = np.zeros(1, np.float32)
    cnt = np.zeros(1, np.uint64)
    _load().orc_value_range(_ptr(x), x.size, _ptr(lo), _ptr(hi), _ptr(cnt))
    return lo[0], hi[0], int(cnt[0])


def eb_params(mode: int, eb: float, vmin=0.0, vmax=0.0, nfinite=0):
    """(eb_abs, h, r) or raises OracleError."""
    e = np.zeros(1, np.float64)
    h = np.zeros(1, np.float32)
    r = np.zeros(1, np.float32)
    st = _load().orc_eb_params(mode, float(eb), float(vmin), float(vmax), int(nfinite), _ptr(e), _ptr(h), _ptr(r))
    if st != OK:
        raise OracleError(st, "eb_params")
    return float(e[0]), np.float32(h[0]), np.float32(r[0])


def prequant(x: np.ndarray, r) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(x.shape, np.int32)
    _load().orc_prequant(_ptr(x), x.size, float(np.float32(r)), _ptr(out))
    return out


def lorenzo_delta(dq: np.ndarray, layers: int = 1) -> np.ndarray:
    """delta = d° - p° per element (row-major, same shape), ndim = dq.ndim,
    with the ``layers``-layer predictor."""
    dq = np.ascontiguousarray(dq, dtype=np.int32)
    out = np.empty(dq.shape, np.int32)
    if layers == 1:
        st = _load().orc_lorenzo_delta(_ptr(dq), dq.ndim, _ptr(_dims(dq.shape)), _ptr(out))
    else:
        st = _load().orc_lorenzo_delta_n(_ptr(dq), dq.ndim, _ptr(_dims(dq.shape)), int(layers), _ptr(out))
    if st != OK:
        raise OracleError(st, "lorenzo_delta")
    return out


def lorenzo_reconstruct(delta: np.ndarray, layers: int = 1) -> np.ndarray:
    delta = np.ascontiguousarray(delta, dtype=np.int32)
    out = np.empty(delta.shape, np.int32)
    if layers == 1:
        st = _load().orc_lorenzo_reconstruct(_ptr(delta), delta.ndim, _ptr(_dims(delta.shape)), _ptr(out))
    else:
        st = _load().orc_lorenzo_reconstruct_n(_ptr(delta), delta.ndim, _ptr(_dims(delta.shape)), int(layers),
                                               _ptr(out))
    if st != OK:
        raise OracleError(st, "lorenzo_reconstruct")
    return out


def huffman_lengths(freq) -> np.ndarray:
    freq = np.ascontiguousarray(np.asarray(freq, dtype=np.uint64))
    out = np.zeros(freq.size, np.uint8)
    m = _load().orc_huffman_lengths(_ptr(freq), freq.size, _ptr(out))
    if m < 0:
        raise OracleError(m, "huffman_lengths")
    return out


def canonical_codes(lengths) -> np.ndarray:
    lengths = np.ascontiguousarray(np.asarray(lengths, dtype=np.uint8))
    out = np.zeros(lengths.size, np.uint64)
    st = _load().orc_canonical_codes(_ptr(lengths), lengths.size, _ptr(out))
    if st != OK:
        raise OracleError(st, "canonical_codes")
    return out


def compress(x: np.ndarray, eb: float, mode: int = EB_VALREL, radius: int = 512,
             sub_size: int = 128, chunk_subs: int = 64, layers: int = 1) -> np.ndarray:
    """Archive bytes (uint8) of ``x`` (float32, 1-3 dims); ``layers`` = 2
    takes the 2-layer Lorenzo predictor (recorded in the header)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32)
    if x.ndim < 1 or x.ndim > 3:
        raise OracleError(EINVAL, "compress: ndim")
    dims = _dims(x.shape)
    size = np.zeros(1, np.uint64)
    if layers == 1:
        st = lib.orc_compressed_size(_ptr(x), x.ndim, _ptr(dims), float(eb), int(mode), radius, sub_size,
                                     chunk_subs, _ptr(size))
    else:
        dummy = np.zeros(1, np.uint8)
        st = lib.orc_compress_layers(_ptr(x), x.ndim, _ptr(dims), float(eb), int(mode), radius, sub_size,
                                     chunk_subs, int(layers), _ptr(dummy), 0, _ptr(size))
        st = OK if st == ETOOSMALL else st
    if st != OK:
        raise OracleError(st, "compress (size)")
    out = np.zeros(int(size[0]), np.uint8)
    st = lib.orc_compress_layers(_ptr(x), x.ndim, _ptr(dims), float(eb), int(mode), radius, sub_size,
                                 chunk_subs, int(layers), _ptr(out), out.size, _ptr(size))
    if st != OK:
        raise OracleError(st, "compress")
    return out


def header_shape(archive: np.ndarray):
    hdr = np.frombuffer(archive[:HEADER_BYTES].tobytes(), dtype=np.uint8)
    ndim = int(hdr[6])
    dims = np.frombuffer(hdr[8:32].tobytes(), dtype=np.uint64)
    return tuple(int(d) for d in dims[3 - ndim:])


def decompress(archive: np.ndarray) -> np.ndarray:
    archive = np.ascontiguousarray(archive, dtype=np.uint8)
    if archive.size < HEADER_BYTES:
        raise OracleError(ECORRUPT, "decompress")
    shape = header_shape(archive)
    n = int(np.prod(shape, dtype=np.uint64)) if shape else 0
    out = np.zeros(shape, np.float32)
    st = _load().orc_decompress(_ptr(archive), archive.size, _ptr(out), n)
    if st != OK:
        raise OracleError(st, "decompress")
    return out


def stages(x: np.ndarray, eb: float, mode: int = EB_VALREL, radius: int = 512):
    """(dq row-major, codes in stream order, histogram, eb_abs)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    dq = np.empty(x.shape, np.int32)
    codes = np.empty(x.size, np.uint16)
    freq = np.zeros(2 * radius, np.uint64)
    e = np.zeros(1, np.float64)
    st = _load().orc_stages(_ptr(x), x.ndim, _ptr(_dims(x.shape)), float(eb), int(mode), radius,
                            _ptr(dq), _ptr(codes), _ptr(freq), _ptr(e))
    if st != OK:
        raise OracleError(st, "stages")
    return dq, codes, freq, float(e[0])
