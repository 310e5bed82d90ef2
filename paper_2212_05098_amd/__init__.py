"""Validating UTF-8 <-> UTF-16LE transcoding on AMD Instinct MI355X (gfx950).

Thin ctypes binding over libutfx.so (C ABI in include/utfx.h).  Every step of the
computation runs in the library's HIP kernels; this module only marshals pointers
and sizes.  PyTorch supplies device memory and streams.  There is no fallback: if
libutfx.so is missing or cannot be loaded, every call raises.

The operations are those of Clausecker & Lemire, "Transcoding Unicode Characters with
AVX-512 Instructions": validating transcoding that stops at the first encoding error
and reports where (sections 6.4, 7.4), validation alone, and output-length queries.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import NamedTuple, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIBRARY = os.path.join(HERE, "libutfx.so")
HEADER = os.path.join(ROOT, "include", "utfx.h")

OK = 0
E_STRAY_CONT = 1
E_MISSING_CONT = 2
E_OVERLONG = 3
E_TOO_LARGE = 4
E_SURROGATE = 5
E_BAD_BYTE = 6
E_OUTPUT_TOO_SMALL = 16
E_INVALID_ARG = 17
E_DEVICE = 18

OP_UTF8_TO_UTF16 = 0
OP_UTF16_TO_UTF8 = 1
OP_VALIDATE_UTF8 = 2
OP_VALIDATE_UTF16 = 3
OP_LENGTH_UTF8 = 4
OP_LENGTH_UTF16 = 5
OP_BATCH = 6

DIR_8TO16 = 0
DIR_16TO8 = 1
# or-ed into a server request's direction: its payload and output are device memory
SERVER_DEVICE_BUFFERS = 0x100


class CResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("reserved", ctypes.c_uint32),
        ("count", ctypes.c_uint64),
        ("written", ctypes.c_uint64),
    ]


class CStream(ctypes.Structure):
    """utfx_stream: the host-side state of a stream (carried units, offsets, verdict)."""
    _fields_ = [
        ("in_units", ctypes.c_uint64),
        ("out_units", ctypes.c_uint64),
        ("err_offset", ctypes.c_uint64),
        ("format", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("n_carry", ctypes.c_uint32),
        ("finished", ctypes.c_uint32),
        ("carry", ctypes.c_uint8 * 4),
        ("carry_need", ctypes.c_uint8),
        ("carry_out", ctypes.c_uint8),
        ("reserved", ctypes.c_uint16),
    ]


STREAM_UTF8_TO_UTF16LE = 0
STREAM_UTF16LE_TO_UTF8 = 1
STREAM_UTF8_TO_UTF16BE = 2
STREAM_UTF16BE_TO_UTF8 = 3


class Result(NamedTuple):
    status: int
    count: int
    written: int


class UtfxError(RuntimeError):
    pass


def exported_functions():
    """Names of the functions include/utfx.h declares."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(utfx_[a-z0-9_]+)\s*\(", text)))


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    """Load libutfx.so (build it first with paper_2212_05098_amd.build.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBRARY):
        raise UtfxError("libutfx.so is not built (run __graft_entry__.build())")
    # torch ships its own HIP runtime under the same soname as the system one; load it
    # first so that the library and torch share one runtime in the process
    import torch  # noqa: F401

    L = ctypes.CDLL(LIBRARY)
    P = ctypes.c_void_p
    Z = ctypes.c_size_t
    U32 = ctypes.c_uint32
    U64 = ctypes.c_uint64
    I = ctypes.c_int
    sigs = {
        "utfx_create": (I, [ctypes.POINTER(P), P]),
        "utfx_destroy": (None, [P]),
        "utfx_last_error": (ctypes.c_char_p, [P]),
        "utfx_set_stream": (I, [P, P]),
        "utfx_set_kernel_events": (I, [P, P, P]),
        "utfx_set_tuning": (I, [P, I, U32, U32, U32]),
        "utfx_get_tuning": (I, [P, I, ctypes.POINTER(U32), ctypes.POINTER(U32), ctypes.POINTER(U32)]),
        "utfx_set_batch_tuning": (I, [P, U32, U32, U32]),
        "utfx_get_batch_tuning": (I, [P, ctypes.POINTER(U32), ctypes.POINTER(U32), ctypes.POINTER(U32)]),
        "utfx_utf16_length_from_utf8": (CResult, [P, P, Z]),
        "utfx_utf8_length_from_utf16le": (CResult, [P, P, Z]),
        "utfx_validate_utf8": (CResult, [P, P, Z]),
        "utfx_validate_utf16le": (CResult, [P, P, Z]),
        "utfx_utf8_to_utf16le": (CResult, [P, P, Z, P, Z]),
        "utfx_utf16le_to_utf8": (CResult, [P, P, Z, P, Z]),
        "utfx_utf16_length_from_utf8_async": (I, [P, P, Z, P]),
        "utfx_utf8_length_from_utf16le_async": (I, [P, P, Z, P]),
        "utfx_validate_utf8_async": (I, [P, P, Z, P]),
        "utfx_validate_utf16le_async": (I, [P, P, Z, P]),
        "utfx_utf8_to_utf16le_async": (I, [P, P, Z, P, Z, P]),
        "utfx_utf16le_to_utf8_async": (I, [P, P, Z, P, Z, P]),
        "utfx_utf8_to_utf16le_noalloc": (I, [P, Z, P, Z, P, P]),
        "utfx_utf8_length_from_utf16be": (CResult, [P, P, Z]),
        "utfx_validate_utf16be": (CResult, [P, P, Z]),
        "utfx_utf8_to_utf16be": (CResult, [P, P, Z, P, Z]),
        "utfx_utf16be_to_utf8": (CResult, [P, P, Z, P, Z]),
        "utfx_utf8_length_from_utf16be_async": (I, [P, P, Z, P]),
        "utfx_validate_utf16be_async": (I, [P, P, Z, P]),
        "utfx_utf8_to_utf16be_async": (I, [P, P, Z, P, Z, P]),
        "utfx_utf16be_to_utf8_async": (I, [P, P, Z, P, Z, P]),
        "utfx_validate_utf32le": (CResult, [P, P, Z]),
        "utfx_utf8_to_utf32le": (CResult, [P, P, Z, P, Z]),
        "utfx_utf32le_to_utf8": (CResult, [P, P, Z, P, Z]),
        "utfx_validate_utf32le_async": (I, [P, P, Z, P]),
        "utfx_utf8_to_utf32le_async": (I, [P, P, Z, P, Z, P]),
        "utfx_utf32le_to_utf8_async": (I, [P, P, Z, P, Z, P]),
        "utfx_utf16le_to_utf32le": (CResult, [P, P, Z, P, Z]),
        "utfx_utf32le_to_utf16le": (CResult, [P, P, Z, P, Z]),
        "utfx_utf16le_to_utf32le_async": (I, [P, P, Z, P, Z, P]),
        "utfx_utf32le_to_utf16le_async": (I, [P, P, Z, P, Z, P]),
        "utfx_utf16be_to_utf32le": (CResult, [P, P, Z, P, Z]),
        "utfx_utf32le_to_utf16be": (CResult, [P, P, Z, P, Z]),
        "utfx_utf16be_to_utf32le_async": (I, [P, P, Z, P, Z, P]),
        "utfx_utf32le_to_utf16be_async": (I, [P, P, Z, P, Z, P]),
        "utfx_stream_init": (I, [ctypes.POINTER(CStream), I]),
        "utfx_stream_transcode": (CResult, [P, ctypes.POINTER(CStream), P, Z, P, Z, I]),
        "utfx_batch_run": (I, [P, P, Z, P, Z, P, U32, U64, P]),
        "utfx_capture_begin": (I, [P]),
        "utfx_capture_end": (I, [P, ctypes.POINTER(P)]),
        "utfx_graph_launch": (I, [P, P]),
        "utfx_graph_destroy": (None, [P]),
        "utfx_server_create": (I, [ctypes.POINTER(P), P]),
        "utfx_server_destroy": (None, [P]),
        "utfx_server_last_error": (ctypes.c_char_p, [P]),
        "utfx_server_submit": (I, [P, U64, P, U64, U32, P, U64]),
        "utfx_server_progress": (I, [P, P, U32, ctypes.POINTER(U32)]),
        "utfx_server_replay": (I, [P, U32, P, P, P, P, P, P, P, P, ctypes.POINTER(U64)]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _res(r: CResult) -> Result:
    return Result(int(r.status), int(r.count), int(r.written))


def _ptr_len(t, unit: int):
    """(device pointer, length in `unit`-byte code units) of a CUDA tensor."""
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch.Tensor on the GPU")
    if not t.is_cuda:
        raise UtfxError("tensor must live on the GPU (no CPU path)")
    if not t.is_contiguous():
        raise UtfxError("tensor must be contiguous")
    nbytes = t.numel() * t.element_size()
    if nbytes % unit:
        raise UtfxError("tensor byte size is not a multiple of the code unit")
    return t.data_ptr(), nbytes // unit


class Context:
    """One library context bound to a HIP stream (default: torch's current stream)."""

    def __init__(self, stream=None):
        import torch

        self._lib = lib()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        st = self._lib.utfx_create(ctypes.byref(h), ctypes.c_void_p(stream.cuda_stream))
        if st != OK:
            raise UtfxError("utfx_create failed with status %d" % st)
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.utfx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        return self._h

    def last_error(self) -> str:
        return (self._lib.utfx_last_error(self._h) or b"").decode()

    def set_kernel_events(self, start=None, stop=None):
        """Record two torch.cuda.Event objects (enable_timing=True) around the main
        kernel of every following single-buffer call; None, None switches it off.
        start.elapsed_time(stop) is then that kernel's own duration in ms."""
        for e in (start, stop):
            if e is not None and not e.cuda_event:
                e.record()  # torch creates its events lazily, on the first record
        a = ctypes.c_void_p(start.cuda_event) if start is not None else None
        b = ctypes.c_void_p(stop.cuda_event) if stop is not None else None
        st = self._lib.utfx_set_kernel_events(self._h, a, b)
        if st != OK:
            raise UtfxError("utfx_set_kernel_events: status %d" % st)

    def set_tuning(self, op: int, tile_bytes: int, tiles_per_segment: int = 8, wgs_per_cu=None):
        """wgs_per_cu None keeps the current value."""
        if wgs_per_cu is None:
            wgs_per_cu = self.get_tuning(op)[2]
        st = self._lib.utfx_set_tuning(self._h, op, tile_bytes, tiles_per_segment, wgs_per_cu)
        if st != OK:
            raise UtfxError("bad tuning %r" % ((op, tile_bytes, tiles_per_segment, wgs_per_cu),))

    def load_tuning(self, path=None) -> bool:
        """Apply the entry for this GPU (architecture, HIP version, CU count) of a tuning
        cache written by paper_2212_05098_amd.tune (default: the package's
        tune_cache.json).  Returns False if there is none."""
        from paper_2212_05098_amd import tune

        entry = tune.load(path or tune.DEFAULT_CACHE)
        if not entry:
            return False
        for op, (tile, seg, wgs) in entry["ops"].items():
            self.set_tuning(int(op), int(tile), int(seg), int(wgs))
        if entry.get("batch"):
            self.set_batch_tuning(*(int(v) for v in entry["batch"]))
        return True

    def set_batch_tuning(self, wave_max_units: int, large_tiles_per_segment: int, large_wgs_per_cu: int):
        st = self._lib.utfx_set_batch_tuning(self._h, wave_max_units, large_tiles_per_segment, large_wgs_per_cu)
        if st != OK:
            raise UtfxError("bad batch tuning %r" % ((wave_max_units, large_tiles_per_segment, large_wgs_per_cu),))

    def get_batch_tuning(self):
        """(wave_max_units, large_tiles_per_segment, large_wgs_per_cu) of the batched call."""
        a, b, c = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        self._lib.utfx_get_batch_tuning(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        return int(a.value), int(b.value), int(c.value)

    def get_tuning(self, op: int):
        """(tile_bytes, tiles_per_segment, wgs_per_cu) of an operation."""
        t = ctypes.c_uint32()
        s = ctypes.c_uint32()
        w = ctypes.c_uint32()
        self._lib.utfx_get_tuning(self._h, op, ctypes.byref(t), ctypes.byref(s), ctypes.byref(w))
        return int(t.value), int(s.value), int(w.value)

    # ---- synchronous calls ------------------------------------------------------
    def utf16_length_from_utf8(self, src) -> Result:
        p, n = _ptr_len(src, 1)
        return _res(self._lib.utfx_utf16_length_from_utf8(self._h, p, n))

    def utf8_length_from_utf16le(self, src) -> Result:
        p, n = _ptr_len(src, 2)
        return _res(self._lib.utfx_utf8_length_from_utf16le(self._h, p, n))

    def validate_utf8(self, src) -> Result:
        p, n = _ptr_len(src, 1)
        return _res(self._lib.utfx_validate_utf8(self._h, p, n))

    def validate_utf16le(self, src) -> Result:
        p, n = _ptr_len(src, 2)
        return _res(self._lib.utfx_validate_utf16le(self._h, p, n))

    def utf8_to_utf16le(self, src, dst) -> Result:
        p, n = _ptr_len(src, 1)
        q, cap = _ptr_len(dst, 2)
        return _res(self._lib.utfx_utf8_to_utf16le(self._h, p, n, q, cap))

    def utf16le_to_utf8(self, src, dst) -> Result:
        p, n = _ptr_len(src, 2)
        q, cap = _ptr_len(dst, 1)
        return _res(self._lib.utfx_utf16le_to_utf8(self._h, p, n, q, cap))

    # raw-pointer forms (for sub-ranges and misaligned views)
    def raw(self, name: str, *args):
        fn = getattr(self._lib, name)
        r = fn(self._h, *args)
        return _res(r) if isinstance(r, CResult) else int(r)

    # ---- asynchronous calls: result goes to a device tensor of 24 bytes ----------
    def utf8_to_utf16le_async(self, src, dst, d_result) -> int:
        p, n = _ptr_len(src, 1)
        q, cap = _ptr_len(dst, 2)
        return int(self._lib.utfx_utf8_to_utf16le_async(self._h, p, n, q, cap, d_result.data_ptr()))

    def utf16le_to_utf8_async(self, src, dst, d_result) -> int:
        p, n = _ptr_len(src, 2)
        q, cap = _ptr_len(dst, 1)
        return int(self._lib.utfx_utf16le_to_utf8_async(self._h, p, n, q, cap, d_result.data_ptr()))

    def validate_utf8_async(self, src, d_result) -> int:
        p, n = _ptr_len(src, 1)
        return int(self._lib.utfx_validate_utf8_async(self._h, p, n, d_result.data_ptr()))

    def validate_utf16le_async(self, src, d_result) -> int:
        p, n = _ptr_len(src, 2)
        return int(self._lib.utfx_validate_utf16le_async(self._h, p, n, d_result.data_ptr()))

    def utf16_length_from_utf8_async(self, src, d_result) -> int:
        p, n = _ptr_len(src, 1)
        return int(self._lib.utfx_utf16_length_from_utf8_async(self._h, p, n, d_result.data_ptr()))

    def utf8_length_from_utf16le_async(self, src, d_result) -> int:
        p, n = _ptr_len(src, 2)
        return int(self._lib.utfx_utf8_length_from_utf16le_async(self._h, p, n, d_result.data_ptr()))

    # ---- UTF-16BE: the same kernels with byte-swapped 16-bit loads or stores --------
    def utf8_length_from_utf16be(self, src) -> Result:
        p, n = _ptr_len(src, 2)
        return _res(self._lib.utfx_utf8_length_from_utf16be(self._h, p, n))

    def validate_utf16be(self, src) -> Result:
        p, n = _ptr_len(src, 2)
        return _res(self._lib.utfx_validate_utf16be(self._h, p, n))

    def utf8_to_utf16be(self, src, dst) -> Result:
        p, n = _ptr_len(src, 1)
        q, cap = _ptr_len(dst, 2)
        return _res(self._lib.utfx_utf8_to_utf16be(self._h, p, n, q, cap))

    def utf16be_to_utf8(self, src, dst) -> Result:
        p, n = _ptr_len(src, 2)
        q, cap = _ptr_len(dst, 1)
        return _res(self._lib.utfx_utf16be_to_utf8(self._h, p, n, q, cap))

    def utf8_to_utf16be_async(self, src, dst, d_result) -> int:
        p, n = _ptr_len(src, 1)
        q, cap = _ptr_len(dst, 2)
        return int(self._lib.utfx_utf8_to_utf16be_async(self._h, p, n, q, cap, d_result.data_ptr()))

    def utf16be_to_utf8_async(self, src, dst, d_result) -> int:
        p, n = _ptr_len(src, 2)
        q, cap = _ptr_len(dst, 1)
        return int(self._lib.utfx_utf16be_to_utf8_async(self._h, p, n, q, cap, d_result.data_ptr()))

    def validate_utf16be_async(self, src, d_result) -> int:
        p, n = _ptr_len(src, 2)
        return int(self._lib.utfx_validate_utf16be_async(self._h, p, n, d_result.data_ptr()))

    def utf8_length_from_utf16be_async(self, src, d_result) -> int:
        p, n = _ptr_len(src, 2)
        return int(self._lib.utfx_utf8_length_from_utf16be_async(self._h, p, n, d_result.data_ptr()))

    def batch_run(self, in_arena, out_arena, d_items, n_items: int, total_in_units: int, d_results) -> int:
        """Queue a batch (see utfx_batch_run); the arenas are uint8 device tensors."""
        return int(
            self._lib.utfx_batch_run(
                self._h,
                in_arena.data_ptr(),
                in_arena.numel() * in_arena.element_size(),
                out_arena.data_ptr(),
                out_arena.numel() * out_arena.element_size(),
                d_items.data_ptr(),
                n_items,
                total_in_units,
                d_results.data_ptr(),
            )
        )


    # ---- UTF-32LE (int32 tensors)
    def validate_utf32le(self, src) -> Result:
        p, n = _ptr_len(src, 4)
        return _res(self._lib.utfx_validate_utf32le(self._h, p, n))

    def utf8_to_utf32le(self, src, dst) -> Result:
        p, n = _ptr_len(src, 1)
        q, cap = _ptr_len(dst, 4)
        return _res(self._lib.utfx_utf8_to_utf32le(self._h, p, n, q, cap))

    def utf32le_to_utf8(self, src, dst) -> Result:
        p, n = _ptr_len(src, 4)
        q, cap = _ptr_len(dst, 1)
        return _res(self._lib.utfx_utf32le_to_utf8(self._h, p, n, q, cap))

    def validate_utf32le_async(self, src, d_result) -> int:
        p, n = _ptr_len(src, 4)
        return int(self._lib.utfx_validate_utf32le_async(self._h, p, n, d_result.data_ptr()))

    def utf8_to_utf32le_async(self, src, dst, d_result) -> int:
        p, n = _ptr_len(src, 1)
        q, cap = _ptr_len(dst, 4)
        return int(self._lib.utfx_utf8_to_utf32le_async(self._h, p, n, q, cap, d_result.data_ptr()))

    def utf32le_to_utf8_async(self, src, dst, d_result) -> int:
        p, n = _ptr_len(src, 4)
        q, cap = _ptr_len(dst, 1)
        return int(self._lib.utfx_utf32le_to_utf8_async(self._h, p, n, q, cap, d_result.data_ptr()))

    def utf16le_to_utf32le(self, src, dst) -> Result:
        p, n = _ptr_len(src, 2)
        q, cap = _ptr_len(dst, 4)
        return _res(self._lib.utfx_utf16le_to_utf32le(self._h, p, n, q, cap))

    def utf32le_to_utf16le(self, src, dst) -> Result:
        p, n = _ptr_len(src, 4)
        q, cap = _ptr_len(dst, 2)
        return _res(self._lib.utfx_utf32le_to_utf16le(self._h, p, n, q, cap))

    def utf16le_to_utf32le_async(self, src, dst, d_result) -> int:
        p, n = _ptr_len(src, 2)
        q, cap = _ptr_len(dst, 4)
        return int(self._lib.utfx_utf16le_to_utf32le_async(self._h, p, n, q, cap, d_result.data_ptr()))

    def utf32le_to_utf16le_async(self, src, dst, d_result) -> int:
        p, n = _ptr_len(src, 4)
        q, cap = _ptr_len(dst, 2)
        return int(self._lib.utfx_utf32le_to_utf16le_async(self._h, p, n, q, cap, d_result.data_ptr()))

    def utf16be_to_utf32le(self, src, dst) -> Result:
        p, n = _ptr_len(src, 2)
        q, cap = _ptr_len(dst, 4)
        return _res(self._lib.utfx_utf16be_to_utf32le(self._h, p, n, q, cap))

    def utf32le_to_utf16be(self, src, dst) -> Result:
        p, n = _ptr_len(src, 4)
        q, cap = _ptr_len(dst, 2)
        return _res(self._lib.utfx_utf32le_to_utf16be(self._h, p, n, q, cap))

    def utf16be_to_utf32le_async(self, src, dst, d_result) -> int:
        p, n = _ptr_len(src, 2)
        q, cap = _ptr_len(dst, 4)
        return int(self._lib.utfx_utf16be_to_utf32le_async(self._h, p, n, q, cap, d_result.data_ptr()))

    def utf32le_to_utf16be_async(self, src, dst, d_result) -> int:
        p, n = _ptr_len(src, 4)
        q, cap = _ptr_len(dst, 2)
        return int(self._lib.utfx_utf32le_to_utf16be_async(self._h, p, n, q, cap, d_result.data_ptr()))

    # ---- streams
    def open_stream(self, fmt: int) -> "Stream":
        return Stream(self, fmt)

    # ---- HIP graphs
    def capture_begin(self):
        st = self._lib.utfx_capture_begin(self._h)
        if st != OK:
            raise UtfxError("capture_begin: %d %s" % (st, self.last_error()))

    def capture_end(self) -> "Graph":
        g = ctypes.c_void_p()
        st = self._lib.utfx_capture_end(self._h, ctypes.byref(g))
        if st != OK:
            raise UtfxError("capture_end: %d %s" % (st, self.last_error()))
        return Graph(self, g)


class Stream:
    """Input in chunks cut at any unit offset (utfx_stream_init / utfx_stream_transcode):
    the concatenated outputs and the first error equal those of one call on the
    concatenated chunks."""

    def __init__(self, ctx: "Context", fmt: int):
        self.ctx = ctx
        self.state = CStream()
        st = ctx._lib.utfx_stream_init(ctypes.byref(self.state), int(fmt))
        if st != OK:
            raise UtfxError("stream_init: bad format %r" % (fmt,))
        self.in16 = fmt in (STREAM_UTF16LE_TO_UTF8, STREAM_UTF16BE_TO_UTF8)

    def transcode(self, src, dst, final: bool = False) -> Result:
        p, n = _ptr_len(src, 2 if self.in16 else 1)
        q, cap = _ptr_len(dst, 1 if self.in16 else 2)
        return _res(self.ctx._lib.utfx_stream_transcode(self.ctx._h, ctypes.byref(self.state), p, n, q, cap,
                                                        1 if final else 0))

    def raw(self, p, n: int, q, cap: int, final: bool = False) -> Result:
        return _res(self.ctx._lib.utfx_stream_transcode(self.ctx._h, ctypes.byref(self.state), p, n, q, cap,
                                                        1 if final else 0))

    @property
    def n_carry(self) -> int:
        return int(self.state.n_carry)

    @property
    def in_units(self) -> int:
        return int(self.state.in_units)

    @property
    def out_units(self) -> int:
        return int(self.state.out_units)


class Graph:
    """A recorded sequence of calls on a Context (utfx_capture_begin / _end)."""

    def __init__(self, ctx: "Context", handle):
        self._ctx = ctx
        self._h = handle

    def launch(self, stream=None):
        import torch

        s = stream if stream is not None else torch.cuda.current_stream()
        st = self._ctx._lib.utfx_graph_launch(self._h, ctypes.c_void_p(s.cuda_stream))
        if st != OK:
            raise UtfxError("graph launch: %d %s" % (st, self._ctx.last_error()))

    def close(self):
        if self._h:
            self._ctx._lib.utfx_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ServerConfig(ctypes.Structure):
    """utfx_server_config"""
    _fields_ = [
        ("arena_in_bytes", ctypes.c_uint64),
        ("arena_out_bytes", ctypes.c_uint64),
        ("device_cap_bytes", ctypes.c_uint64),
        ("max_items", ctypes.c_uint32),
        ("inflight", ctypes.c_uint32),
    ]


class Completion(ctypes.Structure):
    """utfx_completion"""
    _fields_ = [("tag", ctypes.c_uint64), ("result", CResult)]


class Server:
    """Continuous-batching server (utfx_server_*): host requests in, results and
    outputs back on the host."""

    def __init__(self, arena_in_bytes: int, arena_out_bytes: int, max_items: int = 65536, inflight: int = 2,
                 device_cap_bytes: int = 32 << 30):
        self._lib = lib()
        cfg = ServerConfig(arena_in_bytes, arena_out_bytes, device_cap_bytes, max_items, inflight)
        h = ctypes.c_void_p()
        st = self._lib.utfx_server_create(ctypes.byref(h), ctypes.byref(cfg))
        if st != OK:
            raise UtfxError("utfx_server_create failed with status %d" % st)
        self._h = h
        self.max_items = max_items
        self.inflight = inflight

    def close(self):
        if getattr(self, "_h", None):
            self._lib.utfx_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return (self._lib.utfx_server_last_error(self._h) or b"").decode()

    def submit(self, tag: int, data_ptr: int, len_units: int, direction: int, out_ptr: int, out_cap: int) -> int:
        return int(self._lib.utfx_server_submit(self._h, tag, data_ptr, len_units, direction, out_ptr, out_cap))

    def progress(self, max_done: int = 4096):
        """Completions [(tag, Result)] reported by one progress call."""
        buf = (Completion * max_done)()
        n = ctypes.c_uint32()
        st = self._lib.utfx_server_progress(self._h, buf, max_done, ctypes.byref(n))
        if st != OK:
            raise UtfxError("progress: %d %s" % (st, self.last_error()))
        return [(int(buf[i].tag), _res(buf[i].result)) for i in range(n.value)]

    def replay(self, arrival_ns, data_ptrs, len_units, dirs, out_ptrs, out_caps):
        """Real-time replay of an arrival trace (numpy arrays).  Returns (latency_ns
        array, list of Result, wall_ns)."""
        import numpy as np

        n = len(arrival_ns)
        arr = np.ascontiguousarray(arrival_ns, dtype=np.uint64)
        dp = np.ascontiguousarray(data_ptrs, dtype=np.uint64)
        ln = np.ascontiguousarray(len_units, dtype=np.uint64)
        dr = np.ascontiguousarray(dirs, dtype=np.uint32)
        op = np.ascontiguousarray(out_ptrs, dtype=np.uint64)
        oc = np.ascontiguousarray(out_caps, dtype=np.uint64)
        lat = np.zeros(n, dtype=np.uint64)
        res = np.zeros(n * 24, dtype=np.uint8)
        wall = ctypes.c_uint64()
        st = self._lib.utfx_server_replay(self._h, n, arr.ctypes.data, dp.ctypes.data, ln.ctypes.data,
                                          dr.ctypes.data, op.ctypes.data, oc.ctypes.data, lat.ctypes.data,
                                          res.ctypes.data, ctypes.byref(wall))
        if st != OK:
            raise UtfxError("replay: %d %s" % (st, self.last_error()))
        rec = np.dtype([("status", "<i4"), ("reserved", "<u4"), ("count", "<u8"), ("written", "<u8")])
        r = res.view(rec)
        return lat, r, int(wall.value)


# numpy layout of utfx_item (include/utfx.h)
ITEM_FIELDS = [("in_off", "<u8"), ("in_len", "<u8"), ("out_off", "<u8"), ("out_cap", "<u8"), ("dir", "<u4"),
               ("pad", "<u4")]


def pack_items(in_off, in_len, out_off, out_cap, dirs, device="cuda"):
    """Item table for batch_run: a uint8 tensor of len(in_off) utfx_item records."""
    import numpy as np
    import torch

    a = np.zeros(len(in_off), dtype=np.dtype(ITEM_FIELDS))
    a["in_off"], a["in_len"], a["out_off"], a["out_cap"], a["dir"] = in_off, in_len, out_off, out_cap, dirs
    t = torch.from_numpy(a.view(np.uint8).copy())
    return t.to(device) if device else t


def results_from_tensor(t) -> list:
    """Decode a device or host tensor of utfx_result records (24 bytes each)."""
    import numpy as np

    b = t.detach().cpu().contiguous().view(-1).numpy().view(np.uint8)
    rec = np.dtype([("status", "<i4"), ("reserved", "<u4"), ("count", "<u8"), ("written", "<u8")])
    a = b.view(rec)
    return [Result(int(x["status"]), int(x["count"]), int(x["written"])) for x in a]


def result_tensor(n: int = 1, device="cuda"):
    """Device buffer for n utfx_result records."""
    import torch

    return torch.zeros(n * 24, dtype=torch.uint8, device=device)


NOALLOC_MAX_BYTES = (1 << 29) - 32


def utf8_to_utf16le_noalloc(src, dst, d_result, stream=None) -> int:
    """utfx_utf8_to_utf16le_noalloc: the asynchronous UTF-8 -> UTF-16LE call without a
    context or any allocation, on `stream` (default: torch's current stream).  Returns
    the status of queueing it; the result goes to the device tensor d_result."""
    import torch

    p, n = _ptr_len(src, 1)
    q, cap = _ptr_len(dst, 2)
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(lib().utfx_utf8_to_utf16le_noalloc(p, n, q, cap, d_result.data_ptr(), ctypes.c_void_p(s.cuda_stream)))


_default_ctx: Optional[Context] = None


def default_context() -> Context:
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context()
    return _default_ctx


def utf16_length_from_utf8(src) -> Result:
    return default_context().utf16_length_from_utf8(src)


def utf8_length_from_utf16le(src) -> Result:
    return default_context().utf8_length_from_utf16le(src)


def validate_utf8(src) -> Result:
    return default_context().validate_utf8(src)


def validate_utf16le(src) -> Result:
    return default_context().validate_utf16le(src)


def utf8_to_utf16le(src, dst=None):
    """Returns (Result, dst).  dst defaults to n words (always large enough)."""
    import torch

    if dst is None:
        dst = torch.empty(max(src.numel() * src.element_size(), 1), dtype=torch.int16, device=src.device)
    return default_context().utf8_to_utf16le(src, dst), dst


def utf16le_to_utf8(src, dst=None):
    """Returns (Result, dst).  dst defaults to 3n bytes (always large enough)."""
    import torch

    if dst is None:
        n = (src.numel() * src.element_size()) // 2
        dst = torch.empty(max(3 * n, 1), dtype=torch.uint8, device=src.device)
    return default_context().utf16le_to_utf8(src, dst), dst


def utf8_length_from_utf16be(src) -> Result:
    return default_context().utf8_length_from_utf16be(src)


def validate_utf16be(src) -> Result:
    return default_context().validate_utf16be(src)


def utf8_to_utf16be(src, dst=None):
    """Returns (Result, dst).  dst defaults to n words (always large enough)."""
    import torch

    if dst is None:
        dst = torch.empty(max(src.numel() * src.element_size(), 1), dtype=torch.int16, device=src.device)
    return default_context().utf8_to_utf16be(src, dst), dst


def utf16be_to_utf8(src, dst=None):
    """Returns (Result, dst).  dst defaults to 3n bytes (always large enough)."""
    import torch

    if dst is None:
        n = (src.numel() * src.element_size()) // 2
        dst = torch.empty(max(3 * n, 1), dtype=torch.uint8, device=src.device)
    return default_context().utf16be_to_utf8(src, dst), dst
