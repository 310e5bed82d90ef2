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


def build(force: bool = False) -> str:
    """Compile utf_oracle.c into liboracle_utf.so next to it (gcc, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, _SRC]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        path = build()
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


# Exposed for the header-consistency test only.
HEADER = os.path.join(_HERE, "utf_oracle.h")
SOURCE = _SRC
LIBRARY = _LIB
_ = os  # keep flake quiet about re-exports
