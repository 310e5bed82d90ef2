"""Scalar CPU oracle for validating UTF-8 <-> UTF-16LE (and UTF-16BE, UTF-32LE) transcoding.

TEST INFRASTRUCTURE ONLY.  The test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  The GPU library never
imports, links or runs anything in this directory, and this directory never
imports the GPU library.

The arithmetic lives in ``utf_oracle.c`` (plain C, one character at a time, from
the definitions in sections 2.1, 2.2, Table 1, Figure 1(a) and the validation rules
of section 6.4 of Clausecker & Lemire).  This module only builds it with gcc and
marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import NamedTuple, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "utf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_utf.so")

# Separate copy of the status codes (the GPU library has its own in include/utfx.h;
# a test checks that the two agree).
OK = 0
E_STRAY_CONT = 1
E_MISSING_CONT = 2
E_OVERLONG = 3
E_TOO_LARGE = 4
E_SURROGATE = 5
E_BAD_BYTE = 6
E_OUTPUT_TOO_SMALL = 16
E_INVALID_ARG = 17

STATUS_NAMES = {
    OK: "OK",
    E_STRAY_CONT: "STRAY_CONT",
    E_MISSING_CONT: "MISSING_CONT",
    E_OVERLONG: "OVERLONG",
    E_TOO_LARGE: "TOO_LARGE",
    E_SURROGATE: "SURROGATE",
    E_BAD_BYTE: "BAD_BYTE",
    E_OUTPUT_TOO_SMALL: "OUTPUT_TOO_SMALL",
    E_INVALID_ARG: "INVALID_ARG",
}


class _CResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("reserved", ctypes.c_uint32),
        ("count", ctypes.c_uint64),
        ("written", ctypes.c_uint64),
    ]


class Result(NamedTuple):
    status: int
    count: int
    written: int


_TIMING_SRC = os.path.join(_HERE, "oracle_timing.c")
_HDR = os.path.join(_HERE, "utf_oracle.h")


def build(force: bool = False, sanitize: bool = False, lib_path: Optional[str] = None) -> str:
    """Compile utf_oracle.c (strict C99) and the timing harness oracle_timing.c into
    liboracle_utf.so next to them (gcc, -O2).  sanitize builds a separate copy with
    AddressSanitizer and UndefinedBehaviorSanitizer (host code only) at lib_path."""
    out = lib_path or _LIB
    srcs = (_SRC, _TIMING_SRC, _HDR)
    if force or sanitize or not os.path.exists(out) or any(os.path.getmtime(out) < os.path.getmtime(s) for s in srcs):
        tmp = out + ".tmp%d" % os.getpid()
        san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"] if sanitize else []
        objs = []
        for src, std in ((_SRC, "-std=c99"), (_TIMING_SRC, "-std=gnu99")):
            obj = tmp + "." + os.path.basename(src) + ".o"
            subprocess.check_call(["gcc", "-O2", std, "-Wall", "-Wextra", "-fPIC", "-pthread"] + san +
                                  ["-c", "-o", obj, src])
            objs.append(obj)
        subprocess.check_call(["gcc", "-shared", "-pthread"] + san + ["-o", tmp] + objs)
        for o in objs:
            os.remove(o)
        os.replace(tmp, out)
    return out


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        # UTFX_ORACLE_LIB: an already built copy to load instead (the sanitizer test
        # points it at the AddressSanitizer / UndefinedBehaviorSanitizer build)
        path = os.environ.get("UTFX_ORACLE_LIB") or build()
        L = ctypes.CDLL(path)
        p8 = ctypes.c_void_p
        sz = ctypes.c_size_t
        for name, args in [
            ("utfx_ref_utf16_length_from_utf8", [p8, sz]),
            ("utfx_ref_utf8_length_from_utf16le", [p8, sz]),
            ("utfx_ref_validate_utf8", [p8, sz]),
            ("utfx_ref_validate_utf16le", [p8, sz]),
            ("utfx_ref_utf8_to_utf16le", [p8, sz, p8, sz]),
            ("utfx_ref_utf16le_to_utf8", [p8, sz, p8, sz]),
            ("utfx_ref_validate_utf32le", [p8, sz]),
            ("utfx_ref_utf8_to_utf32le", [p8, sz, p8, sz]),
            ("utfx_ref_utf32le_to_utf8", [p8, sz, p8, sz]),
            ("utfx_ref_utf16le_to_utf32le", [p8, sz, p8, sz]),
            ("utfx_ref_utf32le_to_utf16le", [p8, sz, p8, sz]),
        ]:
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = _CResult
        for name in ("utfx_ref_validate_utf8_fixed", "utfx_ref_validate_utf16le_fixed"):
            fn = getattr(L, name)
            fn.argtypes = [p8, sz, sz, p8, p8]
            fn.restype = ctypes.c_uint64
        for name in ("utfx_ref_utf8_to_utf16le_fixed", "utfx_ref_utf16le_to_utf8_fixed"):
            fn = getattr(L, name)
            fn.argtypes = [p8, sz, sz, p8, p8, p8]
            fn.restype = ctypes.c_uint64
        L.utfx_ref_batch.argtypes = [p8, sz, p8, sz, p8, sz, p8]
        L.utfx_ref_batch.restype = ctypes.c_uint64
        ci = ctypes.c_int
        L.utfx_ref_time_buffer.argtypes = [ci, p8, sz, p8, sz, ci, ci, p8, p8, p8, p8, p8]
        L.utfx_ref_time_buffer.restype = ci
        L.utfx_ref_time_batch.argtypes = [p8, sz, p8, sz, p8, sz, p8, ci, ci, p8, p8, p8]
        L.utfx_ref_time_batch.restype = ci
        _lib = L
    return _lib


def _u8(a) -> np.ndarray:
    if isinstance(a, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(a), dtype=np.uint8)
    a = np.ascontiguousarray(a)
    assert a.dtype == np.uint8, a.dtype
    return a


def _u16(a) -> np.ndarray:
    if isinstance(a, (bytes, bytearray, memoryview)):
        b = bytes(a)
        assert len(b) % 2 == 0
        return np.frombuffer(b, dtype="<u2").astype(np.uint16)
    a = np.ascontiguousarray(a)
    assert a.dtype == np.uint16, a.dtype
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data if a.size else None


def _res(r: _CResult) -> Result:
    return Result(int(r.status), int(r.count), int(r.written))


def utf16_length_from_utf8(data) -> Result:
    a = _u8(data)
    return _res(lib().utfx_ref_utf16_length_from_utf8(_ptr(a), a.size))


def utf8_length_from_utf16le(data) -> Result:
    a = _u16(data)
    return _res(lib().utfx_ref_utf8_length_from_utf16le(_ptr(a), a.size))


def validate_utf8(data) -> Result:
    a = _u8(data)
    return _res(lib().utfx_ref_validate_utf8(_ptr(a), a.size))


def validate_utf16le(data) -> Result:
    a = _u16(data)
    return _res(lib().utfx_ref_validate_utf16le(_ptr(a), a.size))


def utf8_to_utf16le(data, cap: Optional[int] = None):
    """Returns (Result, out) where out is a uint16 array of length cap (default n)."""
    a = _u8(data)
    cap = a.size if cap is None else int(cap)
    out = np.zeros(cap, dtype=np.uint16)
    r = _res(lib().utfx_ref_utf8_to_utf16le(_ptr(a), a.size, _ptr(out), cap))
    return r, out


def utf16le_to_utf8(data, cap: Optional[int] = None):
    """Returns (Result, out) where out is a uint8 array of length cap (default 3n)."""
    a = _u16(data)
    cap = 3 * a.size if cap is None else int(cap)
    out = np.zeros(cap, dtype=np.uint8)
    r = _res(lib().utfx_ref_utf16le_to_utf8(_ptr(a), a.size, _ptr(out), cap))
    return r, out


# ---- UTF-16BE (section 2: the same code units, most significant byte first) --------
# A UTF-16BE buffer is handled as the uint16 array that holds its bytes in memory; on
# a little-endian host each element is then the byte-swapped code unit, so these
# wrappers swap every element and defer to the functions above.

def _be_words(data) -> np.ndarray:
    if isinstance(data, (bytes, bytearray, memoryview)):
        b = bytes(data)
        assert len(b) % 2 == 0
        return np.frombuffer(b, dtype=">u2").astype(np.uint16)
    return _u16(data).byteswap()


def utf8_length_from_utf16be(data) -> Result:
    return utf8_length_from_utf16le(_be_words(data))


def validate_utf16be(data) -> Result:
    return validate_utf16le(_be_words(data))


def utf8_to_utf16be(data, cap: Optional[int] = None):
    """Returns (Result, out): out holds the UTF-16BE bytes as a uint16 array."""
    r, out = utf8_to_utf16le(data, cap)
    return r, out.byteswap()


def utf16be_to_utf8(data, cap: Optional[int] = None):
    return utf16le_to_utf8(_be_words(data), cap)


# ---- UTF-32LE (section 2: one 32-bit integer per character) ------------------------

def _u32(a) -> np.ndarray:
    if isinstance(a, (bytes, bytearray, memoryview)):
        b = bytes(a)
        assert len(b) % 4 == 0
        return np.frombuffer(b, dtype="<u4").astype(np.uint32)
    a = np.ascontiguousarray(a)
    assert a.dtype == np.uint32, a.dtype
    return a


def validate_utf32le(data) -> Result:
    a = _u32(data)
    return _res(lib().utfx_ref_validate_utf32le(_ptr(a), a.size))


def utf8_to_utf32le(data, cap: Optional[int] = None):
    """Returns (Result, out) where out is a uint32 array of length cap (default n)."""
    a = _u8(data)
    cap = a.size if cap is None else int(cap)
    out = np.zeros(cap, dtype=np.uint32)
    r = _res(lib().utfx_ref_utf8_to_utf32le(_ptr(a), a.size, _ptr(out), cap))
    return r, out


def utf32le_to_utf8(data, cap: Optional[int] = None):
    """Returns (Result, out) where out is a uint8 array of length cap (default 4n)."""
    a = _u32(data)
    cap = 4 * a.size if cap is None else int(cap)
    out = np.zeros(cap, dtype=np.uint8)
    r = _res(lib().utfx_ref_utf32le_to_utf8(_ptr(a), a.size, _ptr(out), cap))
    return r, out


def utf16le_to_utf32le(data, cap: Optional[int] = None):
    """Returns (Result, out) where out is a uint32 array of length cap (default n)."""
    a = _u16(data)
    cap = a.size if cap is None else int(cap)
    out = np.zeros(cap, dtype=np.uint32)
    r = _res(lib().utfx_ref_utf16le_to_utf32le(_ptr(a), a.size, _ptr(out), cap))
    return r, out


def utf32le_to_utf16le(data, cap: Optional[int] = None):
    """Returns (Result, out) where out is a uint16 array of length cap (default 2n)."""
    a = _u32(data)
    cap = 2 * a.size if cap is None else int(cap)
    out = np.zeros(cap, dtype=np.uint16)
    r = _res(lib().utfx_ref_utf32le_to_utf16le(_ptr(a), a.size, _ptr(out), cap))
    return r, out


def utf16be_to_utf32le(data, cap: Optional[int] = None):
    return utf16le_to_utf32le(_be_words(data), cap)


def utf32le_to_utf16be(data, cap: Optional[int] = None):
    """Returns (Result, out): out holds the UTF-16BE bytes as a uint16 array."""
    r, out = utf32le_to_utf16le(data, cap)
    return r, out.byteswap()


def validate_utf8_fixed(buf: np.ndarray, length: int, want_arrays: bool = True):
    """Validate back-to-back strings of `length` bytes.  Returns (n_valid, status, count)."""
    a = _u8(buf)
    n = a.size // length if length else 0
    st = np.empty(n, dtype=np.int32) if want_arrays else None
    ct = np.empty(n, dtype=np.uint64) if want_arrays else None
    nv = lib().utfx_ref_validate_utf8_fixed(
        _ptr(a), n, length, _ptr(st) if want_arrays else None, _ptr(ct) if want_arrays else None
    )
    return int(nv), st, ct


def validate_utf16le_fixed(buf: np.ndarray, length: int, want_arrays: bool = True):
    a = _u16(buf)
    n = a.size // length if length else 0
    st = np.empty(n, dtype=np.int32) if want_arrays else None
    ct = np.empty(n, dtype=np.uint64) if want_arrays else None
    nv = lib().utfx_ref_validate_utf16le_fixed(
        _ptr(a), n, length, _ptr(st) if want_arrays else None, _ptr(ct) if want_arrays else None
    )
    return int(nv), st, ct


def transcode_fixed(buf: np.ndarray, length: int, utf16_in: bool = False, out=None):
    """Transcode back-to-back strings of `length` units (UTF-8 -> UTF-16LE, or UTF-16LE
    -> UTF-8 with utf16_in), outputs discarded.  Returns (n_valid, status, count,
    written); `out` may supply the three arrays (int32, uint64, uint64, contiguous)."""
    a = _u16(buf) if utf16_in else _u8(buf)
    n = a.size // length if length else 0
    if out is None:
        st = np.empty(n, dtype=np.int32)
        ct = np.empty(n, dtype=np.uint64)
        wr = np.empty(n, dtype=np.uint64)
    else:
        st, ct, wr = out
        assert st.dtype == np.int32 and ct.dtype == wr.dtype == np.uint64 and min(st.size, ct.size, wr.size) >= n
        assert st.flags.c_contiguous and ct.flags.c_contiguous and wr.flags.c_contiguous
    fn = lib().utfx_ref_utf16le_to_utf8_fixed if utf16_in else lib().utfx_ref_utf8_to_utf16le_fixed
    nv = fn(_ptr(a), n, length, _ptr(st), _ptr(ct), _ptr(wr))
    return int(nv), st, ct, wr


# ---- batches: each item is the single-string call on its bytes --------------------

ITEM_DTYPE = np.dtype([("in_off", "<u8"), ("in_len", "<u8"), ("out_off", "<u8"), ("out_cap", "<u8"),
                       ("dir", "<u4"), ("pad", "<u4")])
RESULT_DTYPE = np.dtype([("status", "<i4"), ("reserved", "<u4"), ("count", "<u8"), ("written", "<u8")])


def items_array(in_off, in_len, out_off, out_cap, dirs) -> np.ndarray:
    """A structured array of batch items (the oracle's own copy of the layout)."""
    n = len(in_off)
    it = np.zeros(n, dtype=ITEM_DTYPE)
    it["in_off"], it["in_len"], it["out_off"], it["out_cap"], it["dir"] = in_off, in_len, out_off, out_cap, dirs
    return it


def batch(in_arena: np.ndarray, items: np.ndarray, out_bytes: int):
    """Runs every item (dir 0: UTF-8 -> UTF-16LE, 1: UTF-16LE -> UTF-8) on its bytes.
    Returns (results, out_arena, n_ok): a RESULT_DTYPE array, the uint8 output arena of
    out_bytes bytes (zero outside what the items stored) and the number of OK items."""
    a = _u8(in_arena)
    items = np.ascontiguousarray(items, dtype=ITEM_DTYPE)
    res = np.zeros(items.size, dtype=RESULT_DTYPE)
    out = np.zeros(int(out_bytes), dtype=np.uint8)
    ok = lib().utfx_ref_batch(_ptr(a), a.size, _ptr(out), out.size, _ptr(items), items.size, _ptr(res))
    return res, out, int(ok)


# ---- timing harness of the CPU baseline (oracle_timing.c) --------------------------

TIME_U8_TO_U16, TIME_U16_TO_U8, TIME_VALIDATE_U8, TIME_VALIDATE_U16 = 0, 1, 2, 3


class Timing(NamedTuple):
    seconds: float            # fastest repetition
    threads: int
    result: Result            # combined over the pieces
    out: Optional[np.ndarray]  # transcodes: the pieces' outputs joined in order


def time_buffer(op: int, data, threads: int = 1, reps: int = 3) -> Timing:
    """Fastest of `reps` runs (after one warm-up run) of one oracle operation over the
    buffer on `threads` pinned threads (0 = every CPU of the affinity mask), the input
    cut at character boundaries; steady clock inside C."""
    in16 = op in (TIME_U16_TO_U8, TIME_VALIDATE_U16)
    a = _u16(data) if in16 else _u8(data)
    n = a.size
    if op == TIME_U8_TO_U16:
        out = np.zeros(max(n, 1), dtype=np.uint16)
    elif op == TIME_U16_TO_U8:
        out = np.zeros(max(3 * n, 1), dtype=np.uint8)
    else:
        out = None
    ns = ctypes.c_uint64()
    r = _CResult()
    used = ctypes.c_int()
    lo = np.zeros(256, dtype=np.uint64)
    wr = np.zeros(256, dtype=np.uint64)
    rc = lib().utfx_ref_time_buffer(op, _ptr(a), n, None if out is None else out.ctypes.data,
                                    0 if out is None else (n if op == TIME_U8_TO_U16 else 3 * n), threads, reps,
                                    ctypes.byref(ns), ctypes.byref(r), ctypes.byref(used), lo.ctypes.data,
                                    wr.ctypes.data)
    if rc != 0:
        raise ValueError("bad timing arguments")
    joined = None
    if out is not None:
        scale = 1 if op == TIME_U8_TO_U16 else 3
        # pieces after the first erroring one are not part of the result
        joined = np.concatenate([out[scale * int(lo[k]):scale * int(lo[k]) + int(wr[k])]
                                 for k in range(used.value)])[: r.written] if n else out[:0]
    return Timing(ns.value * 1e-9, used.value, _res(r), joined)


def time_batch(in_arena: np.ndarray, items: np.ndarray, out_bytes: int, threads: int = 1, reps: int = 3):
    """Fastest of `reps` runs (after a warm-up) of the batched reference over the items,
    split into runs of consecutive items of about equal bytes over `threads` pinned
    threads.  Returns (seconds, threads_used, results, n_ok)."""
    a = _u8(in_arena)
    items = np.ascontiguousarray(items, dtype=ITEM_DTYPE)
    res = np.zeros(items.size, dtype=RESULT_DTYPE)
    out = np.zeros(int(out_bytes), dtype=np.uint8)
    ns = ctypes.c_uint64()
    used = ctypes.c_int()
    ok = ctypes.c_uint64()
    rc = lib().utfx_ref_time_batch(_ptr(a), a.size, _ptr(out), out.size, _ptr(items), items.size, _ptr(res),
                                   threads, reps, ctypes.byref(ns), ctypes.byref(used), ctypes.byref(ok))
    if rc != 0:
        raise ValueError("bad timing arguments")
    return ns.value * 1e-9, used.value, res, int(ok.value)


# Exposed for the header-consistency test only.
HEADER = os.path.join(_HERE, "utf_oracle.h")
SOURCE = _SRC
LIBRARY = _LIB
_ = os  # keep flake quiet about re-exports
