"""Pins of the scalar CPU oracle against things other than itself.

Every check here compares the oracle with something it shares no code with: values
the paper prints (tests/golden, each with its citation), CPython's strict codecs (an
independent library implementation of the same standard), closed-form counts of
valid strings, and brute force built from Python's per-character encodings.
"""
import numpy as np
import pytest

import oracle as O
from conftest import read_golden
from paper_2212_05098_amd import synth

STATUS = {v: k for k, v in O.STATUS_NAMES.items()}


def hx(s):
    return [int(t, 16) for t in s.split()]


def all_scalar_values_str():
    cps = np.concatenate([np.arange(0, 0xD800), np.arange(0xE000, 0x110000)]).astype(np.uint32)
    assert cps.size == 1_112_064
    return synth.cps_to_str(cps)


# ------------------------------------------------------------------ paper's printed values

def test_fig1b_codepoints():
    """Figure 1(b): the printed UTF-16 and UTF-8 forms of eight boundary code points."""
    rows = read_golden("fig1b_codepoints.txt")
    assert len(rows) == 8
    for cp_s, u16_s, u8_s in rows:
        u8 = bytes(hx(u8_s))
        u16 = np.array(hx(u16_s), dtype=np.uint16)
        r, out = O.utf8_to_utf16le(u8)
        assert r == O.Result(O.OK, u16.size, u16.size), cp_s
        assert list(out[: r.written]) == list(u16), cp_s
        r, out = O.utf16le_to_utf8(u16)
        assert r == O.Result(O.OK, len(u8), len(u8)), cp_s
        assert bytes(out[: r.written]) == u8, cp_s
        assert O.validate_utf8(u8).status == O.OK
        assert O.validate_utf16le(u16).status == O.OK
        assert O.utf16_length_from_utf8(u8).count == u16.size
        assert O.utf8_length_from_utf16le(u16).count == len(u8)


def test_worked_examples():
    """The opening example of section 6 and the example of section 6.2 print both
    forms; the section 6.1 mask examples print the bytes only (Python supplies the
    words there)."""
    rows = read_golden("worked_examples.txt")
    assert len(rows) == 4
    for label, u8_s, u16_s in rows:
        u8 = bytes(hx(u8_s))
        if u16_s == "-":
            u16 = np.frombuffer(u8.decode("utf-8").encode("utf-16-le"), dtype="<u2")
        else:
            u16 = np.array(hx(u16_s), dtype=np.uint16)
        r, out = O.utf8_to_utf16le(u8)
        assert r.status == O.OK and list(out[: r.written]) == list(u16), label
        r, out = O.utf16le_to_utf8(u16)
        assert r.status == O.OK and bytes(out[: r.written]) == u8, label


def test_sec62_prefix_of_worked_example():
    """Section 6.2: with only the first four bytes of "±1=𝒪" complete, three words are
    produced from four bytes (the straddling 4-byte character is not)."""
    u8 = bytes(hx("C2 B1 31 3D F0 9D 92 AA"))
    r, out = O.utf8_to_utf16le(u8[:4])
    assert r == O.Result(O.OK, 3, 3)
    assert list(out[:3]) == [0x00B1, 0x0031, 0x003D]
    # cut inside the 4-byte character: an error at its lead, with the 3 words before it
    for cut in (5, 6, 7):
        r, out = O.utf8_to_utf16le(u8[:cut])
        assert r == O.Result(O.E_MISSING_CONT, 4, 3)
        assert list(out[:3]) == [0x00B1, 0x0031, 0x003D]


def test_rule_table():
    """Section 6.4 rules 1-6 and the surrogate sequencing rule (sections 2.1, 7.4)."""
    rows = read_golden("rules.txt")
    assert len(rows) >= 30
    for d, units, st, cnt in rows:
        want = O.Result(STATUS[st], int(cnt), int(cnt))
        if d == "u8":
            data = bytes(hx(units))
            assert O.validate_utf8(data) == want, units
            r, _ = O.utf8_to_utf16le(data)
            assert r.status == want.status and (r.status == O.OK or r.count == want.count), units
        else:
            data = np.array(hx(units), dtype=np.uint16)
            assert O.validate_utf16le(data) == want, units
            r, _ = O.utf16le_to_utf8(data)
            assert r.status == want.status and (r.status == O.OK or r.count == want.count), units


# ------------------------------------------------------------------ every scalar value

def test_all_scalar_values_against_python_codecs():
    """All 1,112,064 scalar values in one buffer, both directions, against CPython."""
    s = all_scalar_values_str()
    u8 = np.frombuffer(s.encode("utf-8"), dtype=np.uint8)
    u16 = np.frombuffer(s.encode("utf-16-le"), dtype="<u2").astype(np.uint16)
    # 128 + 1920 + 61440 + 1048576 = 1,112,064 characters; byte and word totals:
    assert u8.size == 128 * 1 + 1920 * 2 + 61440 * 3 + 1048576 * 4
    assert u16.size == (128 + 1920 + 61440) + 2 * 1048576
    r, out = O.utf8_to_utf16le(u8)
    assert r == O.Result(O.OK, u16.size, u16.size)
    assert np.array_equal(out[: r.written], u16)
    r, out = O.utf16le_to_utf8(u16)
    assert r == O.Result(O.OK, u8.size, u8.size)
    assert np.array_equal(out[: r.written], u8)
    assert O.utf16_length_from_utf8(u8).count == u16.size
    assert O.utf8_length_from_utf16le(u16).count == u8.size
    assert O.validate_utf8(u8) == O.Result(O.OK, u8.size, u8.size)
    assert O.validate_utf16le(u16) == O.Result(O.OK, u16.size, u16.size)


def test_utf16be_against_python_codecs():
    """UTF-16BE (section 2, bytes of each code unit in the other order): all scalar
    values against CPython's utf-16-be codec both ways, and every string of length <= 4
    over the 12 representative words against its strict decoder's verdict and offset."""
    s = all_scalar_values_str()
    u8 = np.frombuffer(s.encode("utf-8"), dtype=np.uint8)
    be = s.encode("utf-16-be")
    words = np.frombuffer(be, dtype=np.uint16)  # the buffer as it sits in memory
    r, out = O.utf8_to_utf16be(u8)
    assert r == O.Result(O.OK, words.size, words.size)
    assert out[: r.written].tobytes() == be
    r, out = O.utf16be_to_utf8(words)
    assert r == O.Result(O.OK, u8.size, u8.size)
    assert np.array_equal(out[: r.written], u8)
    assert O.utf8_length_from_utf16be(words).count == u8.size
    assert O.validate_utf16be(words) == O.Result(O.OK, words.size, words.size)
    assert O.utf16be_to_utf8(be)[0] == O.Result(O.OK, u8.size, u8.size)
    for L in range(1, 5):
        strs = _all_strings(ALPHA16, L).astype(np.uint16)
        for i in range(strs.shape[0]):
            b = strs[i].astype(">u2").tobytes()
            try:
                b.decode("utf-16-be")
                want = (O.OK, L)
            except UnicodeDecodeError as e:
                want = (O.E_SURROGATE, e.start // 2)
            got = O.validate_utf16be(np.frombuffer(b, dtype=np.uint16))
            assert (got.status, got.count) == want, strs[i]


ALPHA32 = np.array([0x0, 0x7F, 0x80, 0x7FF, 0x800, 0xD7FF, 0xD800, 0xDBFF, 0xDC00, 0xDFFF, 0xE000, 0xFFFF,
                    0x10000, 0x10FFFF, 0x110000, 0xFFFFFFFF], dtype=np.uint32)


def test_utf32le_against_python_codecs():
    """UTF-32LE (section 2: one 32-bit integer per character): every scalar value against
    CPython's utf-32-le codec both ways; every string of length <= 3 over 16 edge units
    (both surrogate edges, U+10FFFF, the first value past it, 0xFFFFFFFF) against its
    strict decoder's verdict and offset; UTF-8 -> UTF-32 errors at validate_utf8's
    offsets with the valid prefix's characters written."""
    s = all_scalar_values_str()
    u8 = np.frombuffer(s.encode("utf-8"), dtype=np.uint8)
    u32 = np.frombuffer(s.encode("utf-32-le"), dtype="<u4").astype(np.uint32)
    assert u32.size == 1_112_064
    r, out = O.utf8_to_utf32le(u8)
    assert r == O.Result(O.OK, u32.size, u32.size) and np.array_equal(out[: r.written], u32)
    r, out = O.utf32le_to_utf8(u32)
    assert r == O.Result(O.OK, u8.size, u8.size) and np.array_equal(out[: r.written], u8)
    assert O.validate_utf32le(u32) == O.Result(O.OK, u32.size, u32.size)
    for L in range(1, 4):
        strs = _all_strings(ALPHA32, L).astype(np.uint32)
        for i in range(strs.shape[0]):
            b = strs[i].astype("<u4").tobytes()
            try:
                b.decode("utf-32-le")
                want = (O.OK, L)
            except UnicodeDecodeError as e:
                want = (O.E_SURROGATE if 0xD800 <= strs[i][e.start // 4] <= 0xDFFF else O.E_TOO_LARGE, e.start // 4)
            got = O.validate_utf32le(strs[i])
            assert (got.status, got.count) == want, strs[i]
            r, out = O.utf32le_to_utf8(strs[i])
            prefix = b[: 4 * want[1]].decode("utf-32-le").encode("utf-8")
            if want[0] == O.OK:
                assert r == O.Result(O.OK, len(prefix), len(prefix))
            else:
                assert (r.status, r.count) == want
            assert r.written == len(prefix) and out[: r.written].tobytes() == prefix
    rng = synth.rng_for(98, 32)
    for _ in range(300):
        inj = synth.inject_utf8("mixed4", 400, 1e-2, rng)
        v = O.validate_utf8(inj.data)
        r, out = O.utf8_to_utf32le(inj.data)
        prefix = inj.data[: v.count].tobytes().decode("utf-8")
        assert r.status == v.status and r.count == (v.count if v.status else len(prefix))
        assert r.written == len(prefix)
        assert np.array_equal(out[: r.written], np.array([ord(ch) for ch in prefix], np.uint32))


def test_utf16_utf32_against_python_codecs():
    """UTF-16LE <-> UTF-32LE: every scalar value both ways against CPython's codecs;
    every UTF-16 string of length <= 5 over the 12 edge words and every UTF-32 string of
    length <= 3 over the 16 edge units against the strict decoders' verdict and offset,
    with the valid prefix transcoded."""
    s = all_scalar_values_str()
    u16 = np.frombuffer(s.encode("utf-16-le"), dtype="<u2").astype(np.uint16)
    u32 = np.frombuffer(s.encode("utf-32-le"), dtype="<u4").astype(np.uint32)
    r, out = O.utf16le_to_utf32le(u16)
    assert r == O.Result(O.OK, u32.size, u32.size) and np.array_equal(out[: r.written], u32)
    r, out = O.utf32le_to_utf16le(u32)
    assert r == O.Result(O.OK, u16.size, u16.size) and np.array_equal(out[: r.written], u16)
    be = s.encode("utf-16-be")
    r, out = O.utf32le_to_utf16be(u32)
    assert r == O.Result(O.OK, u16.size, u16.size) and out[: r.written].tobytes() == be
    r, out = O.utf16be_to_utf32le(np.frombuffer(be, dtype=np.uint16))
    assert r == O.Result(O.OK, u32.size, u32.size) and np.array_equal(out[: r.written], u32)
    for L in range(1, 6):
        strs = _all_strings(ALPHA16, L).astype(np.uint16)
        for i in range(strs.shape[0]):
            b = strs[i].astype("<u2").tobytes()
            try:
                b.decode("utf-16-le")
                good = L
            except UnicodeDecodeError as e:
                good = e.start // 2
            pre = np.frombuffer(b[: 2 * good].decode("utf-16-le").encode("utf-32-le"), "<u4")
            r, out = O.utf16le_to_utf32le(strs[i])
            if good == L:
                assert r == O.Result(O.OK, pre.size, pre.size)
            else:
                assert (r.status, r.count) == (O.E_SURROGATE, good)
            assert r.written == pre.size and np.array_equal(out[: r.written], pre)
    for L in range(1, 4):
        strs = _all_strings(ALPHA32, L).astype(np.uint32)
        for i in range(strs.shape[0]):
            b = strs[i].astype("<u4").tobytes()
            try:
                b.decode("utf-32-le")
                good = L
            except UnicodeDecodeError as e:
                good = e.start // 4
            pre = np.frombuffer(b[: 4 * good].decode("utf-32-le").encode("utf-16-le"), "<u2")
            r, out = O.utf32le_to_utf16le(strs[i])
            if good == L:
                assert r == O.Result(O.OK, pre.size, pre.size)
            else:
                bad = strs[i][good]
                assert (r.status, r.count) == (O.E_SURROGATE if 0xD800 <= bad <= 0xDFFF else O.E_TOO_LARGE, good)
            assert r.written == pre.size and np.array_equal(out[: r.written], pre)


def test_encoded_surrogates_rejected():
    """Rule 6: the 2,048 surrogate code points in 3-byte form (built by Python's
    surrogatepass handler) are each a SURROGATE error at offset 0."""
    for cp in range(0xD800, 0xE000):
        b = chr(cp).encode("utf-8", "surrogatepass")
        assert O.validate_utf8(b) == O.Result(O.E_SURROGATE, 0, 0), hex(cp)


# ------------------------------------------------------------------ exhaustive and closed forms

def count_valid_utf8(L):
    """Closed form: a valid string of length L ends in a 1-, 2-, 3- or 4-byte
    character, of which there are 128, 1920, 61440 and 1048576."""
    V = [1]
    for k in range(1, L + 1):
        V.append(sum(c * V[k - j] for j, c in ((1, 128), (2, 1920), (3, 61440), (4, 1048576)) if k - j >= 0))
    return V[L]


def test_closed_form_counts():
    assert [count_valid_utf8(L) for L in range(5)] == [1, 128, 18304, 2650112, 383270912]


def _valid_sets_from_python():
    """Valid 1/2/3-byte strings as integer sets, built by concatenating CPython's
    encodings of single characters (brute force, no decoding logic)."""
    by_len = {1: [], 2: [], 3: []}
    for cp in list(range(0, 0xD800)) + list(range(0xE000, 0x10000)):
        b = chr(cp).encode("utf-8")
        by_len[len(b)].append(int.from_bytes(b, "big"))
    e1 = np.array(by_len[1], dtype=np.int64)
    e2 = np.array(by_len[2], dtype=np.int64)
    e3 = np.array(by_len[3], dtype=np.int64)
    V1 = np.zeros(1 << 8, dtype=bool)
    V1[e1] = True
    V2 = np.zeros(1 << 16, dtype=bool)
    V2[e2] = True
    V2[(e1[:, None] << 8 | e1[None, :]).ravel()] = True
    V3 = np.zeros(1 << 24, dtype=bool)
    V3[e3] = True
    V3[(e1[:, None] << 16 | e2[None, :]).ravel()] = True
    V3[(e2[:, None] << 8 | e1[None, :]).ravel()] = True
    t = (e1[:, None] << 8 | e1[None, :]).ravel()
    V3[(t[:, None] << 8 | e1[None, :]).ravel()] = True
    return V1, V2, V3


def test_exhaustive_utf8_up_to_3_bytes():
    """All 16,843,008 byte strings of length <= 3: the oracle's valid set equals the
    brute-force set, the counts equal the closed form, and every first-error offset
    equals the length of the longest valid prefix."""
    V1, V2, V3 = _valid_sets_from_python()
    assert (V1.sum(), V2.sum(), V3.sum()) == (128, 18304, 2650112)
    # length 1
    buf = np.arange(256, dtype=np.uint8)
    nv, st, ct = O.validate_utf8_fixed(buf, 1)
    assert nv == 128 and np.array_equal(st == O.OK, V1)
    assert np.array_equal(ct, np.where(V1, 1, 0))
    # length 2
    x = np.arange(1 << 16, dtype=np.uint32)
    buf = np.stack([(x >> 8) & 0xFF, x & 0xFF], axis=1).astype(np.uint8).ravel()
    nv, st, ct = O.validate_utf8_fixed(buf, 2)
    assert nv == 18304 and np.array_equal(st == O.OK, V2)
    want = np.where(V2, 2, np.where(V1[x >> 8], 1, 0))
    assert np.array_equal(ct, want)
    # length 3
    x = np.arange(1 << 24, dtype=np.uint32)
    buf = np.stack([(x >> 16) & 0xFF, (x >> 8) & 0xFF, x & 0xFF], axis=1).astype(np.uint8).ravel()
    nv, st, ct = O.validate_utf8_fixed(buf, 3)
    assert nv == 2650112 and np.array_equal(st == O.OK, V3)
    want = np.where(V3, 3, np.where(V2[x >> 8], 2, np.where(V1[x >> 16], 1, 0)))
    assert np.array_equal(ct, want)


def test_exhaustive_utf16_one_and_two_words():
    """All 65,536 single words (63,488 valid), and every pair whose first word lies in
    U+D700..E0FF (covering all surrogate interactions): 512 non-surrogates times 63,488
    plus 1,024 highs times 1,024 lows = 2**25 valid pairs."""
    w = np.arange(1 << 16, dtype=np.uint16)
    nv, st, _ = O.validate_utf16le_fixed(w, 1)
    assert nv == 63488
    total = 0
    for first in range(0xD700, 0xE100, 256):
        a = np.repeat(np.arange(first, first + 256, dtype=np.uint32), 1 << 16)
        b = np.tile(np.arange(1 << 16, dtype=np.uint32), 256)
        buf = np.stack([a, b], axis=1).astype(np.uint16).ravel()
        n, _, _ = O.validate_utf16le_fixed(buf, 2, want_arrays=False)
        total += n
    assert total == 512 * 63488 + 1024 * 1024 == 1 << 25


ALPHA8 = [0x00, 0x7F, 0x80, 0x8F, 0x90, 0x9F, 0xA0, 0xBF, 0xC0, 0xC1, 0xC2, 0xDF, 0xE0, 0xE1,
          0xEC, 0xED, 0xEE, 0xEF, 0xF0, 0xF1, 0xF3, 0xF4, 0xF5, 0xF7, 0xF8, 0xFF]
ALPHA16 = [0x0000, 0x007F, 0x0080, 0x07FF, 0x0800, 0xD7FF, 0xD800, 0xDBFF, 0xDC00, 0xDFFF,
           0xE000, 0xFFFF]


def _all_strings(alpha, L):
    idx = np.indices([len(alpha)] * L).reshape(L, -1).T
    return np.array(alpha)[idx]


def test_class_alphabet_utf8_vs_python():
    """Every string of length <= 4 over 26 representative bytes (one per class edge):
    validity and first-error offset equal CPython's strict decoder (error start)."""
    for L in range(1, 5):
        strs = _all_strings(ALPHA8, L).astype(np.uint8)
        nv, st, ct = O.validate_utf8_fixed(strs.ravel(), L)
        for i in range(strs.shape[0]):
            b = strs[i].tobytes()
            try:
                b.decode("utf-8")
                want = (True, L)
            except UnicodeDecodeError as e:
                want = (False, e.start)
            assert (st[i] == O.OK, int(ct[i])) == want, b.hex()


def test_class_alphabet_utf16_vs_python():
    """Every string of length <= 5 over 12 representative words, against CPython's
    strict UTF-16LE decoder (whose error start is in bytes: divided by 2)."""
    for L in range(1, 6):
        strs = _all_strings(ALPHA16, L).astype(np.uint16)
        nv, st, ct = O.validate_utf16le_fixed(strs.ravel(), L)
        for i in range(strs.shape[0]):
            b = strs[i].astype("<u2").tobytes()
            try:
                b.decode("utf-16-le")
                want = (True, L)
            except UnicodeDecodeError as e:
                want = (False, e.start // 2)
            assert (st[i] == O.OK, int(ct[i])) == want, strs[i]


def test_random_3byte_and_4byte_strings_vs_python():
    rng = synth.rng_for(99, 1)
    for L in (3, 4, 7, 16):
        strs = rng.integers(0, 256, size=(40000, L), dtype=np.uint8)
        # bias towards structured bytes: half of the bytes from the class alphabet
        mask = rng.random(strs.shape) < 0.5
        strs[mask] = np.array(ALPHA8, dtype=np.uint8)[rng.integers(0, len(ALPHA8), size=mask.sum())]
        _, st, ct = O.validate_utf8_fixed(strs.ravel(), L)
        for i in range(strs.shape[0]):
            b = strs[i].tobytes()
            try:
                b.decode("utf-8")
                want = (True, L)
            except UnicodeDecodeError as e:
                want = (False, e.start)
            assert (st[i] == O.OK, int(ct[i])) == want, b.hex()


# ------------------------------------------------------------------ invariants

def _check_invariants_u8(data):
    v = O.validate_utf8(data)
    r, out = O.utf8_to_utf16le(data)
    assert r.status == v.status and (r.status == O.OK or r.count == v.count)
    prefix = data[: r.count] if r.status != O.OK else data
    assert O.utf16_length_from_utf8(prefix).count == r.written
    ref = bytes(prefix).decode("utf-8").encode("utf-16-le")
    assert np.array_equal(out[: r.written], np.frombuffer(ref, dtype="<u2"))
    r2, out2 = O.utf8_to_utf16le(prefix)
    assert r2.status == O.OK and np.array_equal(out2[: r2.written], out[: r.written])


def _check_invariants_u16(data):
    v = O.validate_utf16le(data)
    r, out = O.utf16le_to_utf8(data)
    assert r.status == v.status and (r.status == O.OK or r.count == v.count)
    prefix = data[: r.count] if r.status != O.OK else data
    assert O.utf8_length_from_utf16le(prefix).count == r.written
    ref = prefix.astype("<u2").tobytes().decode("utf-16-le").encode("utf-8")
    assert bytes(out[: r.written]) == ref


def test_invariants_on_profiles_and_injections():
    rng = synth.rng_for(7, 7)
    for prof in synth.SCRIPT_PROFILES + ("mixed4",):
        _check_invariants_u8(synth.utf8_buffer(prof, 50_000, rng))
        _check_invariants_u16(synth.utf16_buffer(prof, 25_000, rng))
        for rate in (1e-4, 1e-2):
            inj = synth.inject_utf8(prof, 50_000, rate, rng)
            r = O.validate_utf8(inj.data)
            assert r.status != O.OK and r.count == inj.positions[0]
            _check_invariants_u8(inj.data)
            inj = synth.inject_utf16(prof, 25_000, rate, rng)
            r = O.validate_utf16le(inj.data)
            assert r.status == O.E_SURROGATE and r.count == inj.positions[0]
            _check_invariants_u16(inj.data)


def test_round_trip_config1():
    u8 = synth.config1_buffer()
    assert u8.size == 65536
    r, u16 = O.utf8_to_utf16le(u8)
    assert r.status == O.OK
    r2, back = O.utf16le_to_utf8(u16[: r.written])
    assert r2 == O.Result(O.OK, 65536, 65536)
    assert np.array_equal(back[:65536], u8)
    assert bytes(u8).decode("utf-8").encode("utf-16-le") == u16[: r.written].astype("<u2").tobytes()


# ------------------------------------------------------------------ capacity and edge cases

def test_empty_and_capacity():
    assert O.validate_utf8(b"") == O.Result(O.OK, 0, 0)
    assert O.validate_utf16le(np.zeros(0, np.uint16)) == O.Result(O.OK, 0, 0)
    r, _ = O.utf8_to_utf16le(b"", cap=0)
    assert r == O.Result(O.OK, 0, 0)
    data = "aé€😀".encode("utf-8")  # 1 + 1 + 1 + 2 words
    for cap in range(0, 5):
        r, out = O.utf8_to_utf16le(data, cap=cap)
        assert r == O.Result(O.E_OUTPUT_TOO_SMALL, 5, 0)
    r, out = O.utf8_to_utf16le(data, cap=5)
    assert r == O.Result(O.OK, 5, 5)
    w = np.frombuffer("aé€😀".encode("utf-16-le"), dtype="<u2").astype(np.uint16)
    for cap in range(0, 10):
        r, out = O.utf16le_to_utf8(w, cap=cap)
        assert r == O.Result(O.E_OUTPUT_TOO_SMALL, 10, 0)
    # encoding error outranks a small buffer; nothing stored at or beyond cap
    bad = data + b"\x80"
    r, out = O.utf8_to_utf16le(bad, cap=2)
    assert r == O.Result(O.E_STRAY_CONT, len(data), 5)
    assert out.size == 2


def test_length_formula_upper_bounds_writes():
    """Reading c9: the length query is exact on valid input and an upper bound of
    the units the transcode produces on invalid input."""
    rng = synth.rng_for(5, 5)
    for _ in range(2000):
        b = rng.integers(0, 256, size=int(rng.integers(0, 24)), dtype=np.uint8)
        r, _ = O.utf8_to_utf16le(b, cap=64)
        assert r.written <= O.utf16_length_from_utf8(b).count
        w = rng.choice(np.array(ALPHA16, dtype=np.uint16), size=int(rng.integers(0, 12)))
        r, _ = O.utf16le_to_utf8(w, cap=64)
        assert r.written <= O.utf8_length_from_utf16le(w).count


# ------------------------------------------------------------------ readings of garbled constants

def test_reading_high_surrogate_constant():
    """Reading c10: the footnote's "0xd7c0 = 0xd800 - 0x0020" is a typo; the identity
    that holds for every supplementary code point is hi = (cp >> 10) + 0xD7C0, i.e.
    0xD800 - 0x40.  Checked against Python's UTF-16 encoder."""
    cps = np.arange(0x10000, 0x110000, dtype=np.int64)
    hi = (cps >> 10) + 0xD7C0
    s = synth.cps_to_str(cps.astype(np.uint32))
    w = np.frombuffer(s.encode("utf-16-le"), dtype="<u2").reshape(-1, 2)
    assert np.array_equal(w[:, 0], hi)
    assert 0xD800 - 0xD7C0 == 0x40


def test_reading_surrogate_join_constant():
    """Reading c11: section 7.2's "-0x35f000" is a typo for -0x35F0000 (0xD7C0 << 10);
    the final constant 0xFCA02400 joins every pair: (hi << 10) + lo + 0xFCA02400
    mod 2**32 == code point.  Checked against Python's UTF-16 decoder."""
    hi = np.repeat(np.arange(0xD800, 0xDC00, 4, dtype=np.uint64), 64)
    lo = np.tile(np.arange(0xDC00, 0xE000, 16, dtype=np.uint64), 256)
    joined = ((hi << np.uint64(10)) + lo + np.uint64(0xFCA02400)) & np.uint64(0xFFFFFFFF)
    pairs = np.stack([hi, lo], axis=1).astype("<u2").tobytes().decode("utf-16-le")
    cps = np.frombuffer(pairs.encode("utf-32-le"), dtype="<u4")
    assert np.array_equal(joined.astype(np.uint32), cps)
    assert (-(0xD7C0 << 10) - 0xDC00) % (1 << 32) == 0xFCA02400


# ------------------------------------------------------------------ length query on invalid input

def test_length_query_closed_forms_on_single_units():
    """Reading c9 on every single unit, valid or not.  Over the 256 bytes, Table 1
    gives 128 ASCII bytes (one word each), 64 continuation bytes (none), 32 bytes
    C0..DF and 16 bytes E0..EF (one word each: their characters stay in the BMP) and
    16 bytes F0..FF (two words: a 4-byte character is a surrogate pair, section 6.2):
    128 + 32 + 16 + 2 * 16 = 208.  Over the 65,536 words: 128 below U+0080 (1 byte),
    1,920 below U+0800 (2), 2,048 surrogates (2 each: a pair is 4 bytes, section 7.3)
    and the other 61,440 (3): 192,384."""
    b = np.arange(256, dtype=np.uint8)
    assert O.utf16_length_from_utf8(b) == O.Result(O.OK, 208, 208)
    w = np.arange(65536, dtype=np.uint16)
    assert O.utf8_length_from_utf16le(w) == O.Result(O.OK, 192384, 192384)
    # per unit: a lead byte counts the UTF-16 length of its characters (from CPython's
    # encoder, on the smallest valid character with that lead), a continuation byte 0
    for v in range(256):
        got = O.utf16_length_from_utf8(bytes([v])).count
        if 0x80 <= v <= 0xBF:
            assert got == 0, v
            continue
        ch = None
        for tail in ([], [0x80], [0x80, 0x80], [0x80, 0x80, 0x80], [0xA0, 0x80], [0x90, 0x80, 0x80]):
            try:
                ch = bytes([v] + tail).decode("utf-8")
                break
            except UnicodeDecodeError:
                continue
        if ch is not None and len(ch) == 1:
            assert got == len(ch.encode("utf-16-le")) // 2, v
        else:  # never valid: C0, C1 count as 2-byte leads, F5..FF as 4-byte leads
            assert v in (0xC0, 0xC1) or v >= 0xF5, v
            assert got == (1 if v < 0xF0 else 2), v
    for v in (0x41, 0x7FF, 0x800, 0xD7FF, 0xD800, 0xDBFF, 0xDC00, 0xDFFF, 0xE000, 0xFFFF):
        got = O.utf8_length_from_utf16le(np.array([v], dtype=np.uint16)).count
        if 0xD800 <= v <= 0xDFFF:
            assert got == 2  # half of a 4-byte character
        else:
            assert got == len(chr(v).encode("utf-8")), hex(v)


# ------------------------------------------------------------------ batched reference, timing harness

def test_batch_reference_is_the_single_call_per_item():
    rng = synth.rng_for(31, 1)
    b = synth.make_batch(400, seed_key=(31, 2), median=200, sigma=1.5, hi=20000, err_frac=0.2)
    need = np.where(b.direction == 0, b.in_len, 3 * b.in_len).astype(np.uint64)
    caps = need.copy()
    caps[::7] //= 2  # some outputs too small
    unit = np.where(b.direction == 0, 2, 1).astype(np.uint64)
    out_off = np.concatenate([[0], np.cumsum(caps * unit + 8)[:-1]]).astype(np.uint64)
    out_off += out_off % 2
    dirs = b.direction.copy()
    dirs[5] = 2  # bad direction
    in_off = b.in_off.copy()
    odd = int(np.nonzero(b.direction == 1)[0][0])
    in_off[odd] += 1  # UTF-16 input at an odd offset
    out_bytes = int(out_off[-1] + caps[-1] * unit[-1] + 8)
    items = O.items_array(in_off, b.in_len, out_off, caps, dirs)
    res, out, n_ok = O.batch(b.arena, items, out_bytes)
    assert n_ok == int(np.sum(res["status"] == O.OK))
    for i in range(len(items)):
        if i in (5, odd):
            assert res["status"][i] == O.E_INVALID_ARG
            continue
        a, L, o, cap = int(in_off[i]), int(b.in_len[i]), int(out_off[i]), int(caps[i])
        if dirs[i] == 0:
            want, ref = O.utf8_to_utf16le(b.arena[a:a + L], cap=cap)
            got = out[o:o + 2 * min(want.written, cap)].view(np.uint16)
        else:
            want, ref = O.utf16le_to_utf8(b.arena[a:a + 2 * L].view(np.uint16), cap=cap)
            got = out[o:o + min(want.written, cap)]
        assert (int(res["status"][i]), int(res["count"][i]), int(res["written"][i])) == tuple(want)
        assert np.array_equal(got, ref[:min(want.written, cap)])
    # slots past the arena are refused
    bad = O.items_array([0], [len(b.arena) + 1], [0], [4], [0])
    r, _, _ = O.batch(b.arena, bad, 64)
    assert r["status"][0] == O.E_INVALID_ARG


@pytest.mark.parametrize("threads", [1, 2, 3, 7, 16])
def test_timing_harness_split_matches_one_thread(threads):
    """The CPU baseline's multi-thread split (cuts at character boundaries, results
    combined by the first erroring piece) reproduces the single-call result and output,
    on valid text, on error-dense text and on unpaired surrogates at the cuts."""
    rng = synth.rng_for(32, threads)
    cases8 = [synth.utf8_buffer("mixed4", 100_003, rng),
              synth.inject_utf8("cjk", 50_000, 1e-3, rng).data,
              rng.choice(np.array(ALPHA8, dtype=np.uint8), size=3001)]
    for d in cases8:
        for op in (O.TIME_U8_TO_U16, O.TIME_VALIDATE_U8):
            t = O.time_buffer(op, d, threads=threads, reps=1)
            if op == O.TIME_U8_TO_U16:
                want, ref = O.utf8_to_utf16le(d)
                assert t.result == want, (t.result, want)
                assert np.array_equal(t.out, ref[:want.written])
            else:
                assert t.result == O.validate_utf8(d)
    cases16 = [synth.utf16_buffer("emoji", 60_001, rng),
               synth.inject_utf16("emoji", 40_000, 1e-3, rng).data,
               rng.choice(np.array(ALPHA16, dtype=np.uint16), size=2001)]
    for w in cases16:
        t = O.time_buffer(O.TIME_U16_TO_U8, w, threads=threads, reps=1)
        want, ref = O.utf16le_to_utf8(w)
        assert t.result == want, (t.result, want)
        assert np.array_equal(t.out, ref[:want.written])
        assert O.time_buffer(O.TIME_VALIDATE_U16, w, threads=threads, reps=1).result == O.validate_utf16le(w)
