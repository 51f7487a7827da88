"""Python binding of libdqz (argument marshalling only).

Every function here forwards to the C ABI declared in ``include/dqz.h``; the
compression itself runs in the HIP kernels of ``libdqz.so``.  PyTorch is used
only to own device memory and to name the current HIP stream.  There is no
fallback path: if the library is missing, importing raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdqz.so")

DQZ_OK, DQZ_EINVAL, DQZ_ETOOSMALL, DQZ_ENOMEM, DQZ_ECORRUPT, DQZ_EUNSUPPORTED, DQZ_EHIP = 0, -1, -2, -3, -4, -5, -6
DQZ_EINTERNAL = -7
DQZ_EAGAIN = -8
DQZ_REQ_COMPRESS, DQZ_REQ_DECOMPRESS = 0, 1
DQZ_EB_ABS, DQZ_EB_VALREL = 0, 1
DQZ_HEADER_BYTES = 128
DQZ_DBG_CODES, DQZ_DBG_HISTOGRAM, DQZ_DBG_CODEBOOK, DQZ_DBG_PHASES = 1, 2, 3, 4

DQZ_INJECT_ALLOC_FAIL = 1
DQZ_MAX_LANES = 8
DQZ_LANES_GRAPH = 1
DQZ_TUNE_FORCE = 1

EXPORTED = ("dqz_ctx_create", "dqz_ctx_destroy", "dqz_ctx_reserve", "dqz_ctx_workspace", "dqz_compress_bound",
            "dqz_decompress_bound", "dqz_compress", "dqz_compress_async", "dqz_compress_async_static",
            "dqz_archive_info", "dqz_decompress",
            "dqz_decompress_async", "dqz_status_str", "dqz_ctx_last_error", "dqz_debug_copy", "dqz_debug_inject",
            "dqz_ctx_set_timing", "dqz_stage_times", "dqz_ctx_set_lanes", "dqz_batch_workspace", "dqz_compress_batch",
            "dqz_decompress_batch", "dqz_tune", "dqz_server_create", "dqz_server_destroy", "dqz_server_submit",
            "dqz_server_wait", "dqz_server_get_stats", "dqz_stream_workspace", "dqz_stream_compress", "dqz_stream_info",
            "dqz_stream_decompress")
DQZ_MAX_STAGES = 8
COMPRESS_STAGES = ("init", "range_eb", "quantize", "quantize_scan", "codebook", "encode")
DECOMPRESS_STAGES = ("decode_tables", "inflate", "reconstruct")


def timing_stage(which: int, stage) -> int:
    """Timing level that records only the events around one stage (index or name)."""
    if isinstance(stage, str):
        stage = (COMPRESS_STAGES if which == 0 else DECOMPRESS_STAGES).index(stage)
    return 0x100 | (int(which) << 4) | int(stage)


class DqzError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class dqz_shape(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("dims", ctypes.c_uint64 * 3)]


class dqz_params(ctypes.Structure):
    _fields_ = [("eb", ctypes.c_double), ("eb_mode", ctypes.c_int32), ("radius", ctypes.c_uint32),
                ("sub_size", ctypes.c_uint32), ("chunk_subs", ctypes.c_uint32), ("layers", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class dqz_result(ctypes.Structure):
    """What an _async call reports (written by its kernels)."""
    _fields_ = [("flags", ctypes.c_uint32), ("status", ctypes.c_int32), ("archive_bytes", ctypes.c_uint64),
                ("workspace_need", ctypes.c_uint64), ("reserved", ctypes.c_uint64),
                ("header", ctypes.c_uint8 * DQZ_HEADER_BYTES)]


DQZ_RESULT_BYTES = ctypes.sizeof(dqz_result)


class dqz_server_config(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("workspace_bytes", ctypes.c_uint64),
                ("hbm_budget", ctypes.c_uint64)]


class dqz_request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("d_input", ctypes.c_void_p),
                ("input_bytes", ctypes.c_uint64), ("d_output", ctypes.c_void_p), ("output_capacity", ctypes.c_uint64),
                ("shape", dqz_shape), ("params", dqz_params), ("header", ctypes.c_uint8 * DQZ_HEADER_BYTES)]


class dqz_completion(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("reserved", ctypes.c_uint32), ("output_bytes", ctypes.c_uint64),
                ("footprint", ctypes.c_uint64), ("t_submit_us", ctypes.c_double), ("t_admit_us", ctypes.c_double),
                ("t_done_us", ctypes.c_double), ("header", ctypes.c_uint8 * DQZ_HEADER_BYTES)]


class dqz_server_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("submitted", "admitted", "completed", "failed", "retried",
                                                "max_running", "max_in_flight_bytes")]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libdqz.so is not built ({LIB_PATH}); run __graft_entry__.build()")
    # torch ships its own HIP runtime under the same soname; load it first so
    # that libdqz binds to the runtime that owns the process's device memory
    # and streams (two runtimes in one process cannot share the GPU).
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32
    lib.dqz_ctx_create.argtypes = [ctypes.c_int, u64, ctypes.POINTER(P)]
    lib.dqz_ctx_create.restype = i32
    lib.dqz_ctx_destroy.argtypes = [P]
    lib.dqz_ctx_destroy.restype = None
    lib.dqz_ctx_reserve.argtypes = [P, u64]
    lib.dqz_ctx_reserve.restype = i32
    lib.dqz_ctx_workspace.argtypes = [P, ctypes.POINTER(u64), ctypes.POINTER(u64)]
    lib.dqz_ctx_workspace.restype = i32
    lib.dqz_decompress_bound.argtypes = [P, u64, ctypes.POINTER(u64)]
    lib.dqz_decompress_bound.restype = i32
    lib.dqz_compress_async.argtypes = [P, P, ctypes.POINTER(dqz_shape), ctypes.POINTER(dqz_params), P, u64, P, P]
    lib.dqz_compress_async.restype = i32
    lib.dqz_compress_async_static.argtypes = [P, ctypes.POINTER(dqz_shape), ctypes.POINTER(dqz_params), P, u64, P, P]
    lib.dqz_compress_async_static.restype = i32
    lib.dqz_ctx_set_lanes.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32]
    lib.dqz_ctx_set_lanes.restype = i32
    lib.dqz_batch_workspace.argtypes = [ctypes.c_uint32, ctypes.POINTER(dqz_shape), ctypes.POINTER(dqz_params),
                                        ctypes.c_uint32, ctypes.POINTER(u64)]
    lib.dqz_batch_workspace.restype = i32
    lib.dqz_compress_batch.argtypes = [P, ctypes.c_uint32, ctypes.POINTER(P), ctypes.POINTER(dqz_shape),
                                       ctypes.POINTER(dqz_params), ctypes.POINTER(P), ctypes.POINTER(u64), P, P]
    lib.dqz_compress_batch.restype = i32
    lib.dqz_decompress_batch.argtypes = [P, ctypes.c_uint32, ctypes.POINTER(P), ctypes.POINTER(u64), P,
                                         ctypes.POINTER(P), ctypes.POINTER(u64), P, P]
    lib.dqz_decompress_batch.restype = i32
    lib.dqz_tune.argtypes = [P, P, ctypes.POINTER(dqz_shape), ctypes.POINTER(dqz_params), ctypes.c_double,
                             ctypes.c_uint32, ctypes.POINTER(dqz_params), P]
    lib.dqz_tune.restype = i32
    lib.dqz_stream_workspace.argtypes = [ctypes.POINTER(dqz_shape), ctypes.POINTER(dqz_params), u64,
                                         ctypes.POINTER(u64), ctypes.POINTER(u64)]
    lib.dqz_stream_workspace.restype = i32
    lib.dqz_stream_compress.argtypes = [P, P, ctypes.POINTER(dqz_shape), ctypes.POINTER(dqz_params), u64, P, u64,
                                        ctypes.POINTER(u64), P]
    lib.dqz_stream_compress.restype = i32
    lib.dqz_stream_info.argtypes = [P, u64, ctypes.POINTER(dqz_shape), ctypes.POINTER(ctypes.c_uint32),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(u64)]
    lib.dqz_stream_info.restype = i32
    lib.dqz_stream_decompress.argtypes = [P, P, u64, P, u64, P]
    lib.dqz_stream_decompress.restype = i32
    lib.dqz_server_create.argtypes = [ctypes.c_int, ctypes.POINTER(dqz_server_config), ctypes.POINTER(P)]
    lib.dqz_server_create.restype = i32
    lib.dqz_server_destroy.argtypes = [P]
    lib.dqz_server_destroy.restype = None
    lib.dqz_server_submit.argtypes = [P, ctypes.POINTER(dqz_request), ctypes.POINTER(u64)]
    lib.dqz_server_submit.restype = i32
    lib.dqz_server_wait.argtypes = [P, u64, ctypes.c_int64, ctypes.POINTER(dqz_completion)]
    lib.dqz_server_wait.restype = i32
    lib.dqz_server_get_stats.argtypes = [P, ctypes.POINTER(dqz_server_stats)]
    lib.dqz_server_get_stats.restype = i32
    lib.dqz_decompress_async.argtypes = [P, P, u64, P, P, u64, P, P]
    lib.dqz_decompress_async.restype = i32
    lib.dqz_debug_inject.argtypes = [P, ctypes.c_int, ctypes.c_int]
    lib.dqz_debug_inject.restype = i32
    lib.dqz_compress_bound.argtypes = [ctypes.POINTER(dqz_shape), ctypes.POINTER(dqz_params),
                                       ctypes.POINTER(u64), ctypes.POINTER(u64)]
    lib.dqz_compress_bound.restype = i32
    lib.dqz_compress.argtypes = [P, P, ctypes.POINTER(dqz_shape), ctypes.POINTER(dqz_params), P, u64,
                                 ctypes.POINTER(u64), P, P]
    lib.dqz_compress.restype = i32
    lib.dqz_archive_info.argtypes = [P, u64, ctypes.POINTER(dqz_shape), ctypes.POINTER(dqz_params),
                                     ctypes.POINTER(u64), ctypes.POINTER(u64)]
    lib.dqz_archive_info.restype = i32
    lib.dqz_decompress.argtypes = [P, P, u64, P, P, u64, P]
    lib.dqz_decompress.restype = i32
    lib.dqz_status_str.argtypes = [i32]
    lib.dqz_status_str.restype = ctypes.c_char_p
    lib.dqz_ctx_last_error.argtypes = [P]
    lib.dqz_ctx_last_error.restype = ctypes.c_char_p
    lib.dqz_debug_copy.argtypes = [P, ctypes.c_int, P, u64]
    lib.dqz_debug_copy.restype = i32
    lib.dqz_ctx_set_timing.argtypes = [P, ctypes.c_int]
    lib.dqz_ctx_set_timing.restype = i32
    lib.dqz_stage_times.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
    lib.dqz_stage_times.restype = i32
    return lib


lib = _load()


def make_shape(shape) -> dqz_shape:
    s = dqz_shape()
    s.ndim = len(shape)           # the library rejects ndim outside 1..3
    for i, d in enumerate(list(shape)[:3]):
        s.dims[i] = int(d)
    return s


def make_params(eb: float, mode: int = DQZ_EB_VALREL, radius: int = 0, sub_size: int = 0,
                chunk_subs: int = 0, layers: int = 0) -> dqz_params:
    p = dqz_params()
    p.eb = float(eb)
    p.eb_mode = int(mode)
    p.radius = int(radius)
    p.sub_size = int(sub_size)
    p.chunk_subs = int(chunk_subs)
    p.layers = int(layers)
    return p


def _mode(mode) -> int:
    if isinstance(mode, str):
        return {"abs": DQZ_EB_ABS, "valrel": DQZ_EB_VALREL}[mode]
    return int(mode)


def dqz_compress_bound(shape, params: dqz_params):
    amax, ws = ctypes.c_uint64(0), ctypes.c_uint64(0)
    s = make_shape(shape)
    st = lib.dqz_compress_bound(ctypes.byref(s), ctypes.byref(params), ctypes.byref(amax), ctypes.byref(ws))
    if st != DQZ_OK:
        raise DqzError(st, f"dqz_compress_bound: {lib.dqz_status_str(st).decode()}")
    return int(amax.value), int(ws.value)


def dqz_compress_async_static(field_ptr: int, shape, params: dqz_params, archive_ptr: int, archive_cap: int,
                              result_ptr: int, stream=None) -> int:
    """dqz_compress_async on the library's fixed per-GPU workspace (no context,
    no allocation); the device writes a dqz_result at result_ptr.  `stream`: a
    torch stream of the current device (None: its current stream)."""
    import torch  # streams only
    if stream is None:
        stream = torch.cuda.current_stream()
    s = make_shape(shape)
    return lib.dqz_compress_async_static(ctypes.c_void_p(field_ptr), ctypes.byref(s), ctypes.byref(params),
                                         ctypes.c_void_p(archive_ptr), int(archive_cap), ctypes.c_void_p(result_ptr),
                                         ctypes.c_void_p(stream.cuda_stream))


def dqz_stream_workspace(shape, params: dqz_params, slab_bytes: int):
    """(workspace bytes, largest container) of a streaming compression."""
    ws, cmax = ctypes.c_uint64(0), ctypes.c_uint64(0)
    s = make_shape(shape)
    st = lib.dqz_stream_workspace(ctypes.byref(s), ctypes.byref(params), int(slab_bytes), ctypes.byref(ws),
                                  ctypes.byref(cmax))
    if st != DQZ_OK:
        raise DqzError(st, f"dqz_stream_workspace: {lib.dqz_status_str(st).decode()}")
    return int(ws.value), int(cmax.value)


def _host_ptr(a) -> int:
    """Address of a host buffer: an ndarray (its .ctypes) or a CPU torch tensor."""
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def dqz_stream_info(container):
    """(shape tuple, slabs, absolute bound, workspace bytes) of a container in host memory."""
    s, n, eb, ws = dqz_shape(), ctypes.c_uint32(0), ctypes.c_double(0), ctypes.c_uint64(0)
    nbytes = container.nbytes if hasattr(container, "nbytes") and not hasattr(container, "data_ptr") \
        else container.numel() * container.element_size()
    st = lib.dqz_stream_info(ctypes.c_void_p(_host_ptr(container)), int(nbytes), ctypes.byref(s), ctypes.byref(n),
                             ctypes.byref(eb), ctypes.byref(ws))
    if st != DQZ_OK:
        raise DqzError(st, f"dqz_stream_info: {lib.dqz_status_str(st).decode()}")
    return tuple(int(s.dims[i]) for i in range(s.ndim)), int(n.value), float(eb.value), int(ws.value)


def dqz_decompress_bound(header: bytes) -> int:
    ws = ctypes.c_uint64(0)
    buf = ctypes.create_string_buffer(bytes(header), len(header))
    st = lib.dqz_decompress_bound(buf, len(header), ctypes.byref(ws))
    if st != DQZ_OK:
        raise DqzError(st, f"dqz_decompress_bound: {lib.dqz_status_str(st).decode()}")
    return int(ws.value)


def dqz_archive_info(header: bytes):
    s, p = dqz_shape(), dqz_params()
    n, ab = ctypes.c_uint64(0), ctypes.c_uint64(0)
    buf = ctypes.create_string_buffer(bytes(header), len(header))
    st = lib.dqz_archive_info(buf, len(header), ctypes.byref(s), ctypes.byref(p), ctypes.byref(n), ctypes.byref(ab))
    if st != DQZ_OK:
        raise DqzError(st, f"dqz_archive_info: {lib.dqz_status_str(st).decode()}")
    shape = tuple(int(s.dims[i]) for i in range(s.ndim))
    return shape, p, int(n.value), int(ab.value)


@dataclass
class Compressed:
    """An archive in device memory plus a host copy of its header."""
    archive: "object"        # torch.uint8 CUDA tensor, exactly the archive bytes
    header: bytes            # the 128-byte header

    @property
    def nbytes(self) -> int:
        return int(self.archive.numel())


@dataclass
class BatchBuffers:
    """Archive and result buffers of one batch (see Context.batch_buffers)."""
    shapes: list
    params: list
    archives: list
    results: object


class Context:
    """Owns one dqz_ctx (its device workspace is kept across calls).

    The tensor-level helpers (compress / decompress) reserve the workspace a
    call needs before making it; the raw forwarders do not."""

    def __init__(self, device: int = 0, workspace: int = 0):
        import torch  # device memory and streams only
        self._torch = torch
        self.device = device
        h = ctypes.c_void_p()
        st = lib.dqz_ctx_create(device, int(workspace), ctypes.byref(h))
        if st != DQZ_OK:
            why = lib.dqz_ctx_last_error(None).decode()
            raise DqzError(st, f"dqz_ctx_create: {lib.dqz_status_str(st).decode()} ({why})")
        self.handle = h
        self.lanes = 1

    def dqz_ctx_reserve(self, nbytes: int):
        self._check(lib.dqz_ctx_reserve(self.handle, int(nbytes)), "dqz_ctx_reserve")

    def dqz_ctx_workspace(self):
        """(workspace bytes held, workspace the most recent call needed)"""
        cap, need = ctypes.c_uint64(0), ctypes.c_uint64(0)
        self._check(lib.dqz_ctx_workspace(self.handle, ctypes.byref(cap), ctypes.byref(need)), "dqz_ctx_workspace")
        return int(cap.value), int(need.value)

    def dqz_debug_inject(self, what: int, count: int):
        self._check(lib.dqz_debug_inject(self.handle, int(what), int(count)), "dqz_debug_inject")

    def close(self):
        if getattr(self, "handle", None):
            lib.dqz_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, what: str):
        if st != DQZ_OK:
            msg = lib.dqz_ctx_last_error(self.handle).decode()
            raise DqzError(st, f"{what}: {lib.dqz_status_str(st).decode()} ({msg})")

    def _stream(self, stream):
        torch = self._torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(stream.cuda_stream)

    # -- raw C-ABI forwarding (caller-provided buffers) -------------------------------
    def dqz_compress(self, field_ptr: int, shape, params: dqz_params, archive_ptr: int, archive_cap: int,
                     stream=None):
        """Returns (status, archive_bytes, header bytes)."""
        s = make_shape(shape)
        nbytes = ctypes.c_uint64(0)
        hdr = ctypes.create_string_buffer(DQZ_HEADER_BYTES)
        st = lib.dqz_compress(self.handle, ctypes.c_void_p(field_ptr), ctypes.byref(s), ctypes.byref(params),
                              ctypes.c_void_p(archive_ptr), int(archive_cap), ctypes.byref(nbytes), hdr,
                              self._stream(stream))
        return st, int(nbytes.value), hdr.raw

    def dqz_decompress(self, archive_ptr: int, archive_bytes: int, header: bytes | None, field_ptr: int,
                       field_cap_elems: int, stream=None) -> int:
        hb = ctypes.create_string_buffer(bytes(header), DQZ_HEADER_BYTES) if header is not None else None
        return lib.dqz_decompress(self.handle, ctypes.c_void_p(archive_ptr), int(archive_bytes), hb,
                                  ctypes.c_void_p(field_ptr), int(field_cap_elems), self._stream(stream))

    def dqz_compress_async(self, field_ptr: int, shape, params: dqz_params, archive_ptr: int, archive_cap: int,
                           result_ptr: int, stream=None) -> int:
        """Enqueue only; the device writes a dqz_result at result_ptr."""
        s = make_shape(shape)
        return lib.dqz_compress_async(self.handle, ctypes.c_void_p(field_ptr), ctypes.byref(s), ctypes.byref(params),
                                      ctypes.c_void_p(archive_ptr), int(archive_cap), ctypes.c_void_p(result_ptr),
                                      self._stream(stream))

    def dqz_decompress_async(self, archive_ptr: int, archive_bytes: int, header: bytes, field_ptr: int,
                             field_cap_elems: int, result_ptr: int, stream=None) -> int:
        hb = ctypes.create_string_buffer(bytes(header), DQZ_HEADER_BYTES)
        return lib.dqz_decompress_async(self.handle, ctypes.c_void_p(archive_ptr), int(archive_bytes), hb,
                                        ctypes.c_void_p(field_ptr), int(field_cap_elems),
                                        ctypes.c_void_p(result_ptr), self._stream(stream))

    def dqz_ctx_set_timing(self, level):
        """0 off, 1 (or True) stage events, 2 also the decoding kernel's per-wave phase sums,
        timing_stage(which, stage): the two events around one stage only."""
        self._check(lib.dqz_ctx_set_timing(self.handle, int(level)), "dqz_ctx_set_timing")

    def dqz_stage_times(self, which: int) -> dict:
        """Microseconds per stage of the last timed compress (0) / decompress (1)."""
        us = (ctypes.c_double * DQZ_MAX_STAGES)()
        n = ctypes.c_int(0)
        self._check(lib.dqz_stage_times(self.handle, which, us, ctypes.byref(n)), "dqz_stage_times")
        names = COMPRESS_STAGES if which == 0 else DECOMPRESS_STAGES
        return {names[i]: float(us[i]) for i in range(n.value)}

    def dqz_debug_copy(self, what: int, nbytes: int):
        import numpy as np
        out = np.empty(nbytes, np.uint8)
        st = lib.dqz_debug_copy(self.handle, what, ctypes.c_void_p(out.ctypes.data), nbytes)
        self._check(st, "dqz_debug_copy")
        return out

    # -- tensor-level helpers ---------------------------------------------------------
    def compress(self, field, eb: float, mode="valrel", radius: int = 0, sub_size: int = 0, chunk_subs: int = 0,
                 out=None, stream=None, layers: int = 0) -> Compressed:
        """Compress a float32 CUDA tensor (1-3 dims, contiguous; a 4-dim one
        is compressed as 3D with its two slowest axes merged)."""
        torch = self._torch
        if field.dtype != torch.float32 or not field.is_cuda or not field.is_contiguous():
            raise DqzError(DQZ_EINVAL, "field must be a contiguous float32 CUDA tensor")
        if field.dim() == 4:
            field = field.view(field.shape[0] * field.shape[1], field.shape[2], field.shape[3])
        params = make_params(eb, _mode(mode), radius, sub_size, chunk_subs, layers)
        shape = tuple(field.shape)
        bound, ws = dqz_compress_bound(shape, params)
        self.dqz_ctx_reserve(ws)
        if out is None or out.numel() < bound:
            out = torch.empty(bound, dtype=torch.uint8, device=field.device)
        st, nbytes, hdr = self.dqz_compress(field.data_ptr(), shape, params, out.data_ptr(), out.numel(), stream)
        self._check(st, "dqz_compress")
        return Compressed(out[:nbytes], hdr)

    def decompress(self, comp, out=None, stream=None):
        """Decompress a Compressed (or a uint8 CUDA tensor holding an archive)."""
        torch = self._torch
        if isinstance(comp, Compressed):
            arc, hdr = comp.archive, comp.header
        else:
            arc, hdr = comp, None
        if hdr is None:
            hdr = bytes(arc[:DQZ_HEADER_BYTES].cpu().numpy().tobytes())
        shape, _, n, _ = dqz_archive_info(hdr)
        self.dqz_ctx_reserve(dqz_decompress_bound(hdr))
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=arc.device)
        st = self.dqz_decompress(arc.data_ptr(), arc.numel(), hdr, out.data_ptr(), out.numel(), stream)
        self._check(st, "dqz_decompress")
        return out

    # -- host path ----------------------------------------------------------------------
    def stream_compress(self, x, eb: float, mode="valrel", slab_bytes: int = 256 << 20, out=None, radius: int = 0,
                        sub_size: int = 0, chunk_subs: int = 0, stream=None, layers: int = 0):
        """Compress a host field (C-contiguous float32 numpy array or CPU torch
        tensor, pinned for overlapped copies) slab by slab into a container in
        host memory; returns the container (a prefix view of `out` if given)."""
        import numpy as np
        params = make_params(eb, _mode(mode), radius, sub_size, chunk_subs, layers)
        shape = tuple(x.shape)
        ws, cmax = dqz_stream_workspace(shape, params, slab_bytes)
        self.dqz_ctx_reserve(ws)
        if out is None:
            out = np.empty(cmax, dtype=np.uint8)
        cap = out.nbytes if not hasattr(out, "data_ptr") else out.numel()
        nbytes = ctypes.c_uint64(0)
        st = lib.dqz_stream_compress(self.handle, ctypes.c_void_p(_host_ptr(x)), ctypes.byref(make_shape(shape)),
                                     ctypes.byref(params), int(slab_bytes), ctypes.c_void_p(_host_ptr(out)), int(cap),
                                     ctypes.byref(nbytes), self._stream(stream))
        self._check(st, "dqz_stream_compress")
        return out[:int(nbytes.value)]

    def stream_decompress(self, container, out=None, stream=None):
        """Decompress a container from host memory into a host field (numpy
        float32 unless `out`, a float32 host array or CPU tensor, is given)."""
        import numpy as np
        shape, _, _, ws = dqz_stream_info(container)
        self.dqz_ctx_reserve(ws)
        if out is None:
            out = np.empty(shape, dtype=np.float32)
        cap = out.size if not hasattr(out, "data_ptr") else out.numel()
        nbytes = container.nbytes if not hasattr(container, "data_ptr") else container.numel()
        st = lib.dqz_stream_decompress(self.handle, ctypes.c_void_p(_host_ptr(container)), int(nbytes),
                                       ctypes.c_void_p(_host_ptr(out)), int(cap), self._stream(stream))
        self._check(st, "dqz_stream_decompress")
        return out

    # -- batched calls ------------------------------------------------------------------
    def dqz_ctx_set_lanes(self, lanes: int, flags: int = 0):
        self._check(lib.dqz_ctx_set_lanes(self.handle, int(lanes), int(flags)), "dqz_ctx_set_lanes")
        self.lanes = int(lanes)

    def batch_buffers(self, fields, ebs, mode="valrel", **kw) -> "BatchBuffers":
        """Archive and result buffers for a batch of these fields (reusing them
        keeps a captured batch graph valid across calls)."""
        torch = self._torch
        params = [make_params(eb, _mode(mode), kw.get("radius", 0), kw.get("sub_size", 0), kw.get("chunk_subs", 0),
                              kw.get("layers", 0)) for eb in ebs]
        shapes = [tuple(f.shape) for f in fields]
        caps = [dqz_compress_bound(s, p)[0] for s, p in zip(shapes, params)]
        arcs = [torch.empty(c, dtype=torch.uint8, device=f.device) for c, f in zip(caps, fields)]
        res = torch.zeros(len(fields) * DQZ_RESULT_BYTES, dtype=torch.uint8, device=fields[0].device)
        return BatchBuffers(shapes, params, arcs, res)

    def compress_batch(self, fields, ebs, mode="valrel", buffers=None, reserve=True, stream=None, **kw):
        """Compress several float32 CUDA tensors in one dqz_compress_batch call;
        returns one Compressed per field."""
        torch = self._torch
        n = len(fields)
        for f in fields:
            if f.dtype != torch.float32 or not f.is_cuda or not f.is_contiguous():
                raise DqzError(DQZ_EINVAL, "fields must be contiguous float32 CUDA tensors")
        if buffers is None:
            buffers = self.batch_buffers(fields, ebs, mode, **kw)
        shapes = (dqz_shape * n)(*[make_shape(s) for s in buffers.shapes])
        params = (dqz_params * n)(*buffers.params)
        if reserve:
            lanes = max(1, self.lanes)
            need = ctypes.c_uint64(0)
            st = lib.dqz_batch_workspace(n, shapes, params, lanes, ctypes.byref(need))
            self._check(st, "dqz_batch_workspace")
            self.dqz_ctx_reserve(int(need.value))
        P = ctypes.c_void_p
        fptr = (P * n)(*[f.data_ptr() for f in fields])
        aptr = (P * n)(*[a.data_ptr() for a in buffers.archives])
        caps = (ctypes.c_uint64 * n)(*[a.numel() for a in buffers.archives])
        st = lib.dqz_compress_batch(self.handle, n, fptr, shapes, params, aptr, caps,
                                    P(buffers.results.data_ptr()), self._stream(stream))
        self._check(st, "dqz_compress_batch")
        raw = buffers.results.cpu().numpy().tobytes()      # waits for the batch
        res = [dqz_result.from_buffer_copy(raw[i * DQZ_RESULT_BYTES:(i + 1) * DQZ_RESULT_BYTES]) for i in range(n)]
        short = [r.workspace_need for r in res if r.status == DQZ_ENOMEM]
        if short and reserve:
            # a lane's exception overflow pool was too small: give every lane
            # the largest reported need on top and run the batch again
            self.dqz_ctx_reserve(self.dqz_ctx_workspace()[0] + max(1, self.lanes) * max(short))
            return self.compress_batch(fields, ebs, mode, buffers, False, stream, **kw)
        out = []
        for i, r in enumerate(res):
            if r.status != DQZ_OK:
                raise DqzError(r.status, f"dqz_compress_batch: field {i}: {lib.dqz_status_str(r.status).decode()}")
            out.append(Compressed(buffers.archives[i][:r.archive_bytes], bytes(r.header)))
        return out

    def decompress_batch(self, comps, outs=None, reserve=True, stream=None):
        """Decompress several Compressed archives in one dqz_decompress_batch call."""
        torch = self._torch
        n = len(comps)
        hdrs = b"".join(c.header for c in comps)
        shapes = [dqz_archive_info(c.header)[0] for c in comps]
        if reserve:
            # each lane holds the largest decompression layout of its fields
            need = sum(sorted((dqz_decompress_bound(c.header) for c in comps), reverse=True)[:max(1, self.lanes)])
            self.dqz_ctx_reserve(need)
        if outs is None:
            outs = [torch.empty(s, dtype=torch.float32, device=c.archive.device) for s, c in zip(shapes, comps)]
        P = ctypes.c_void_p
        aptr = (P * n)(*[c.archive.data_ptr() for c in comps])
        abytes = (ctypes.c_uint64 * n)(*[c.archive.numel() for c in comps])
        fptr = (P * n)(*[o.data_ptr() for o in outs])
        fcap = (ctypes.c_uint64 * n)(*[o.numel() for o in outs])
        res = torch.zeros(n * DQZ_RESULT_BYTES, dtype=torch.uint8, device=comps[0].archive.device)
        hb = ctypes.create_string_buffer(hdrs, len(hdrs))
        st = lib.dqz_decompress_batch(self.handle, n, aptr, abytes, hb, fptr, fcap, P(res.data_ptr()),
                                      self._stream(stream))
        if st == DQZ_ENOMEM and reserve:
            self.dqz_ctx_reserve(self.dqz_ctx_workspace()[1])
            st = lib.dqz_decompress_batch(self.handle, n, aptr, abytes, hb, fptr, fcap, P(res.data_ptr()),
                                          self._stream(stream))
        self._check(st, "dqz_decompress_batch")
        raw = res.cpu().numpy().tobytes()
        for i in range(n):
            r = dqz_result.from_buffer_copy(raw[i * DQZ_RESULT_BYTES:(i + 1) * DQZ_RESULT_BYTES])
            if r.status != DQZ_OK:
                raise DqzError(r.status, f"dqz_decompress_batch: archive {i}: {lib.dqz_status_str(r.status).decode()}")
        return outs

    def tune(self, field, eb: float, mode="valrel", radius: int = 0, tolerance: float = 0.05, force: bool = False,
             stream=None) -> dqz_params:
        """dqz_tune: subchunk and chunk sizes for this field's shape class."""
        p = make_params(eb, _mode(mode), radius)
        s = make_shape(tuple(field.shape))
        _, ws = dqz_compress_bound(tuple(field.shape), p)
        amax = dqz_compress_bound(tuple(field.shape), p)[0]
        self.dqz_ctx_reserve(ws + amax + 4 * field.numel() + (64 << 20) + 4096)
        out = dqz_params()
        st = lib.dqz_tune(self.handle, ctypes.c_void_p(field.data_ptr()), ctypes.byref(s), ctypes.byref(p),
                          float(tolerance), DQZ_TUNE_FORCE if force else 0, ctypes.byref(out), self._stream(stream))
        self._check(st, "dqz_tune")
        return out


class Server:
    """One dqz_server: continuous batching of compression and decompression
    requests (marshalling only; admission, launches and completion tracking
    run in the library's dispatcher thread).  Buffers passed to submit_* must
    stay alive until the request is collected with wait()."""

    def __init__(self, device: int = 0, slots: int = 4, workspace: int = 1 << 30, budget: int = 64 << 30):
        cfg = dqz_server_config(int(slots), 0, int(workspace), int(budget))
        h = ctypes.c_void_p()
        st = lib.dqz_server_create(int(device), ctypes.byref(cfg), ctypes.byref(h))
        if st != DQZ_OK:
            raise DqzError(st, f"dqz_server_create: {lib.dqz_status_str(st).decode()}")
        self.handle = h
        self._keep = {}

    def submit_compress(self, field, eb: float, out, mode="valrel", radius: int = 0, sub_size: int = 0,
                        chunk_subs: int = 0, layers: int = 0) -> int:
        r = dqz_request()
        r.kind = DQZ_REQ_COMPRESS
        r.d_input = field.data_ptr()
        r.d_output = out.data_ptr()
        r.output_capacity = out.numel() * out.element_size()
        r.shape = make_shape(tuple(field.shape))
        r.params = make_params(eb, _mode(mode), radius, sub_size, chunk_subs, layers)
        return self._submit(r, (field, out))

    def submit_decompress(self, archive, nbytes: int, header: bytes, out) -> int:
        r = dqz_request()
        r.kind = DQZ_REQ_DECOMPRESS
        r.d_input = archive.data_ptr()
        r.input_bytes = int(nbytes)
        r.d_output = out.data_ptr()
        r.output_capacity = out.numel() * out.element_size()
        ctypes.memmove(r.header, bytes(header), DQZ_HEADER_BYTES)
        return self._submit(r, (archive, out))

    def _submit(self, r, keep) -> int:
        t = ctypes.c_uint64(0)
        st = lib.dqz_server_submit(self.handle, ctypes.byref(r), ctypes.byref(t))
        if st != DQZ_OK:
            raise DqzError(st, f"dqz_server_submit: {lib.dqz_status_str(st).decode()}")
        self._keep[int(t.value)] = keep
        return int(t.value)

    def wait(self, ticket: int, timeout_us: int = -1) -> dqz_completion:
        c = dqz_completion()
        st = lib.dqz_server_wait(self.handle, int(ticket), int(timeout_us), ctypes.byref(c))
        if st != DQZ_OK:
            raise DqzError(st, f"dqz_server_wait: {lib.dqz_status_str(st).decode()}")
        self._keep.pop(int(ticket), None)
        return c

    def stats(self) -> dict:
        s = dqz_server_stats()
        st = lib.dqz_server_get_stats(self.handle, ctypes.byref(s))
        if st != DQZ_OK:
            raise DqzError(st, "dqz_server_get_stats")
        return {k: int(getattr(s, k)) for k, _ in dqz_server_stats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            lib.dqz_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default = {}


def default_context(device: int = 0) -> Context:
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def compress(field, eb: float, mode="valrel", **kw) -> Compressed:
    return default_context(field.device.index or 0).compress(field, eb, mode, **kw)


def decompress(comp, **kw):
    arc = comp.archive if isinstance(comp, Compressed) else comp
    return default_context(arc.device.index or 0).decompress(comp, **kw)
