"""CPU-side checks of the C-ABI library: it builds for gfx950, loads, exports every
function include/utfx.h declares, and its status codes match the oracle's copy.
No compute call is made here (there may be no GPU)."""
import ctypes
import os
import re

import pytest

import paper_2212_05098_amd as utfx
from paper_2212_05098_amd import build as B
import oracle as O


@pytest.fixture(scope="module")
def libpath():
    if not os.path.exists(B.LIB):
        B.build()
    return B.LIB


def test_library_exports_every_declared_function(libpath):
    names = utfx.exported_functions()
    assert len(names) >= 19
    L = ctypes.CDLL(libpath)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_signatures_cover_header(libpath):
    L = utfx.lib()
    for n in utfx.exported_functions():
        assert getattr(L, n).argtypes is not None, n


def _enum(path, prefix):
    text = open(path).read()
    return {m.group(1): int(m.group(2)) for m in re.finditer(r"\b%s([A-Z_]+)\s*=\s*(\d+)" % prefix, text)}


def test_status_codes_match_oracle_copy():
    lib_codes = _enum(os.path.join(os.path.dirname(B.LIB), "..", "include", "utfx.h"), "UTFX_E_")
    lib_codes["OK"] = 0
    ora_codes = _enum(O.HEADER, "UTFX_REF_E_")
    ora_codes["OK"] = 0
    for k, v in ora_codes.items():
        assert lib_codes[k] == v, k
    assert utfx.E_OUTPUT_TOO_SMALL == lib_codes["OUTPUT_TOO_SMALL"]
    assert utfx.E_DEVICE == lib_codes["DEVICE"]


def test_result_struct_layout():
    assert ctypes.sizeof(utfx.CResult) == 24
    assert utfx.CResult.count.offset == 8 and utfx.CResult.written.offset == 16


def test_stream_state_layout_and_init(libpath):
    """utfx_stream matches the header's layout; utfx_stream_init is host-only (it
    launches nothing), zeroes the state and rejects unknown formats and a null state."""
    assert ctypes.sizeof(utfx.CStream) == 48 and utfx.CStream.carry.offset == 40
    L = utfx.lib()
    st = utfx.CStream()
    ctypes.memset(ctypes.byref(st), 0x77, ctypes.sizeof(st))
    assert L.utfx_stream_init(ctypes.byref(st), utfx.STREAM_UTF16BE_TO_UTF8) == utfx.OK
    assert (st.in_units, st.out_units, st.err_offset, st.status, st.n_carry, st.finished) == (0, 0, 0, 0, 0, 0)
    assert st.format == utfx.STREAM_UTF16BE_TO_UTF8 and bytes(st.carry) == bytes(4)
    assert (st.carry_need, st.carry_out, st.reserved) == (0, 0, 0)
    assert L.utfx_stream_init(ctypes.byref(st), 4) == utfx.E_INVALID_ARG
    assert L.utfx_stream_init(ctypes.byref(st), -1) == utfx.E_INVALID_ARG
    assert L.utfx_stream_init(None, 0) == utfx.E_INVALID_ARG


def test_product_path_never_touches_the_oracle():
    """The library and its binding share nothing with oracle/ and never load it."""
    pkg = os.path.dirname(utfx.__file__)
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")) and f != "synth.py":
                text = open(os.path.join(root, f)).read()
                assert "oracle" not in text.lower(), os.path.join(root, f)
    text = open(os.path.join(pkg, "synth.py")).read()
    assert "import oracle" not in text and "from oracle" not in text


def test_no_cpu_fallback_without_gpu():
    """Without a GPU tensor the binding refuses instead of computing on the host."""
    import torch

    with pytest.raises((utfx.UtfxError, TypeError)):
        utfx._ptr_len(torch.zeros(4, dtype=torch.uint8), 1)


def test_tune_cache_round_trip(tmp_path):
    """The tuning cache is plain JSON that load() returns unchanged."""
    from paper_2212_05098_amd import tune

    entry = {"key": "gfx950|hip x|256 CUs", "device": "x", "size_mib": 1, "ops": {"0": [8192, 4, 4]},
             "batch": [16384, 4, 2]}
    p = str(tmp_path / "c.json")
    tune.save(entry, p)
    assert tune.load(p, key=entry["key"]) == entry
    assert tune.load(str(tmp_path / "missing.json"), key=entry["key"]) is None


def test_header_is_plain_c(tmp_path):
    """include/utfx.h compiles as strict C99 and its structs have the sizes and offsets
    the library and the binding assume."""
    import shutil
    import subprocess

    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(B.LIB), "..", "include")
    src = tmp_path / "h.c"
    src.write_text(
        '#include <stddef.h>\n#include "utfx.h"\n'
        "int main(void) {\n"
        "  return !(sizeof(utfx_result) == 24 && offsetof(utfx_result, count) == 8 &&\n"
        "           sizeof(utfx_stream) == 48 && offsetof(utfx_stream, carry) == 40 &&\n"
        "           offsetof(utfx_stream, carry_need) == 44 && sizeof(utfx_item) == 40);\n"
        "}\n")
    exe = tmp_path / "h"
    subprocess.check_call([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", inc, str(src), "-o",
                           str(exe)])
    assert subprocess.run([str(exe)]).returncode == 0
