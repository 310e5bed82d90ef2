"""UTF-32LE through the C ABI against the oracle (pinned to CPython's utf-32-le codec):
UTF-8 -> UTF-32 (validation of section 6.4, code points of Figure 1(a)), UTF-32 ->
UTF-8 (section 2's range and surrogate rules) and UTF-16LE <-> UTF-32LE (section 2.1),
element by element, at ragged sizes that span many segments, with injected errors,
every UTF-8 error kind and every unpaired surrogate at every chunk offset, the
class-edge alphabets, misaligned pointers, small outputs, the async forms and one 256
MiB buffer per direction."""
import numpy as np
import pytest

import oracle as O
import paper_2212_05098_amd as utfx
from paper_2212_05098_amd import synth
from gpu_helpers import (check_u16_to_u32, check_u32_to_u16, check_u32_to_u8, check_u8_to_u32, dev_u8, dev_u16,
                         dev_u32, note)

pytestmark = pytest.mark.gpu

SIZES = (1, 2, 3, 5, 15, 16, 17, 63, 64, 65, 1000, 4095, 4096, 4097, 8191, 8193, 16_385, 40_000, 300_007)


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available()
    c = utfx.Context()
    yield c
    c.close()


@pytest.mark.parametrize("prof", synth.SCRIPT_PROFILES + ("mixed4",))
def test_profiles_ragged_sizes(ctx, prof):
    rng = synth.rng_for(80, synth.PROFILE_IDS[prof])
    for n in SIZES:
        note("utf32 %s n=%d" % (prof, n))
        data = synth.utf8_buffer(prof, n, rng)
        check_u8_to_u32(ctx, data)
        check_u32_to_u8(ctx, synth.utf32_buffer(prof, n, rng))


def test_round_trip(ctx):
    import torch

    rng = synth.rng_for(81)
    data = synth.utf8_buffer("mixed4", 2_000_003, rng)
    src, _ = dev_u8(data)
    mid = torch.empty(data.size, dtype=torch.int32, device="cuda")
    r = ctx.utf8_to_utf32le(src, mid)
    assert r.status == utfx.OK
    back = torch.empty(4 * r.written, dtype=torch.uint8, device="cuda")
    r2 = ctx.utf32le_to_utf8(mid[: r.written], back)
    assert r2 == (utfx.OK, data.size, data.size)
    assert np.array_equal(back[: data.size].cpu().numpy(), data)


@pytest.mark.parametrize("prof", ["cjk", "mixed4", "emoji"])
@pytest.mark.parametrize("rate", [1e-4, 3e-2])
def test_injected_errors(ctx, prof, rate):
    rng = synth.rng_for(82, synth.PROFILE_IDS[prof], int(rate * 1e6))
    for trial in range(3):
        inj = synth.inject_utf8(prof, 200_000, rate, rng)
        note("utf32 inject utf8 %s rate=%g trial=%d" % (prof, rate, trial))
        r = check_u8_to_u32(ctx, inj.data)
        assert r.status != utfx.OK and r.count == inj.positions[0]
        units, pos = synth.inject_utf32(synth.utf32_buffer(prof, 100_000, rng), rate, rng)
        note("utf32 inject utf32 %s rate=%g trial=%d" % (prof, rate, trial))
        r = check_u32_to_u8(ctx, units)
        assert r.status in (utfx.E_SURROGATE, utfx.E_TOO_LARGE) and r.count == pos[0]


@pytest.mark.parametrize("kind", synth.UTF8_KINDS)
def test_each_utf8_error_kind_at_every_chunk_offset(ctx, kind):
    rng = synth.rng_for(83, synth.UTF8_KINDS.index(kind))
    base = synth.utf8_buffer("mixed4", 4000, rng).tobytes()
    for off in range(0, 81):
        item = synth.utf8_error_item(kind, rng)
        prefix = base[:off].decode("utf-8", errors="ignore").encode("utf-8")
        prefix += b"a" * (off - len(prefix))
        data = np.frombuffer(prefix + item + b"z" + base[off:], dtype=np.uint8)
        note("utf32 kind %s off=%d" % (kind, off))
        assert check_u8_to_u32(ctx, data).count == off


def test_class_alphabets(ctx):
    from test_oracle_pins import ALPHA8, ALPHA32, _all_strings

    for L in (1, 2, 3):
        strs = _all_strings(ALPHA32, L).astype(np.uint32)
        note("utf32 alphabet L=%d (%d strings)" % (L, strs.shape[0]))
        for s in strs:
            check_u32_to_u8(ctx, s, guard=8)
    for L in (1, 2):
        strs = _all_strings(ALPHA8, L).astype(np.uint8)
        note("utf8->utf32 alphabet L=%d" % L)
        for s in strs:
            check_u8_to_u32(ctx, s, guard=8)


@pytest.mark.parametrize("shift", [0, 1, 2, 3, 5, 7, 13])
def test_misaligned_pointers(ctx, shift):
    rng = synth.rng_for(84, shift)
    data = synth.utf8_buffer("mixed4", 20_011, rng)
    units = synth.utf32_buffer("emoji", 10_007, rng)
    note("utf32 misaligned shift=%d" % shift)
    check_u8_to_u32(ctx, data, in_shift=shift, out_shift=shift % 4)
    check_u32_to_u8(ctx, units, in_shift=shift % 4, out_shift=shift)


def test_output_capacity(ctx):
    rng = synth.rng_for(85)
    data = synth.utf8_buffer("mixed4", 50_000, rng)
    need = O.utf8_to_utf32le(data)[0].count
    for cap in (0, 1, 3, 4, 5, need // 2, need - 1, need):
        note("utf32 cap u8 %d" % cap)
        r = check_u8_to_u32(ctx, data, cap=cap, out_shift=1)
        assert r.status == (utfx.OK if cap >= need else utfx.E_OUTPUT_TOO_SMALL)
    units = synth.utf32_buffer("cjk", 20_000, rng)
    need = O.utf32le_to_utf8(units)[0].count
    for cap in (0, 1, 15, 16, 17, need - 1, need):
        note("utf32 cap u32 %d" % cap)
        r = check_u32_to_u8(ctx, units, cap=cap, out_shift=3)
        assert r.status == (utfx.OK if cap >= need else utfx.E_OUTPUT_TOO_SMALL)
    inj = synth.inject_utf8("cjk", 50_000, 1e-4, rng)
    check_u8_to_u32(ctx, inj.data, cap=10)


def test_empty_and_arguments(ctx):
    import torch

    e8 = torch.zeros(0, dtype=torch.uint8, device="cuda")
    e32 = torch.zeros(0, dtype=torch.int32, device="cuda")
    o32 = torch.zeros(4, dtype=torch.int32, device="cuda")
    o8 = torch.zeros(4, dtype=torch.uint8, device="cuda")
    assert ctx.utf8_to_utf32le(e8, o32) == (utfx.OK, 0, 0)
    assert ctx.utf32le_to_utf8(e32, o8) == (utfx.OK, 0, 0)
    assert ctx.validate_utf32le(e32) == (utfx.OK, 0, 0)
    b = torch.zeros(64, dtype=torch.uint8, device="cuda")
    for off in (1, 2, 3):
        assert ctx.raw("utfx_validate_utf32le", b.data_ptr() + off, 4).status == utfx.E_INVALID_ARG
        assert ctx.raw("utfx_utf32le_to_utf8", b.data_ptr() + off, 4, b.data_ptr(), 16).status == utfx.E_INVALID_ARG
        assert ctx.raw("utfx_utf8_to_utf32le", b.data_ptr(), 4, b.data_ptr() + off, 4).status == utfx.E_INVALID_ARG
    assert ctx.raw("utfx_utf32le_to_utf8", None, 4, b.data_ptr(), 16).status == utfx.E_INVALID_ARG


def test_async_forms(ctx):
    import torch

    rng = synth.rng_for(86)
    data = synth.utf8_buffer("mixed4", 70_001, rng)
    units, pos = synth.inject_utf32(synth.utf32_buffer("emoji", 30_001, rng), 1e-4, rng)
    s8, _ = dev_u8(data)
    s32, _ = dev_u32(units)
    o32 = torch.empty(data.size, dtype=torch.int32, device="cuda")
    o8 = torch.empty(4 * units.size, dtype=torch.uint8, device="cuda")
    res = utfx.result_tensor(3)
    assert ctx.utf8_to_utf32le_async(s8, o32, res[0:24]) == utfx.OK
    assert ctx.utf32le_to_utf8_async(s32, o8, res[24:48]) == utfx.OK
    assert ctx.validate_utf32le_async(s32, res[48:72]) == utfx.OK
    torch.cuda.synchronize()
    got = utfx.results_from_tensor(res)
    w32, r32 = O.utf8_to_utf32le(data)
    w8, r8 = O.utf32le_to_utf8(units)
    assert tuple(got[0]) == tuple(w32)
    assert np.array_equal(o32.cpu().numpy().view(np.uint32)[: w32.written], r32[: w32.written])
    assert tuple(got[1]) == tuple(w8) and w8.count == pos[0]
    assert np.array_equal(o8.cpu().numpy()[: w8.written], r8[: w8.written])
    assert tuple(got[2]) == tuple(O.validate_utf32le(units))


def test_full_size_each_direction(ctx):
    """256 MiB per direction: mixed UTF-8 to UTF-32, and 64 Mi CJK units to UTF-8."""
    import torch

    full = 256 << 20
    data = synth.config_buffer("mixed4", synth.DIR_8TO16, full, config=2)
    note("utf32 full size utf8->utf32")
    r = check_u8_to_u32(ctx, data)
    assert r.status == utfx.OK
    torch.cuda.empty_cache()
    rng = synth.rng_for(87)
    units = synth.utf32_buffer("cjk", full // 4, rng)
    note("utf32 full size utf32->utf8")
    r = check_u32_to_u8(ctx, units)
    assert r.status == utfx.OK
    torch.cuda.empty_cache()


# ---------------------------------------------------------------- UTF-16LE <-> UTF-32LE

@pytest.mark.parametrize("prof", synth.SCRIPT_PROFILES + ("mixed4",))
def test_utf16_utf32_ragged_sizes(ctx, prof):
    rng = synth.rng_for(90, synth.PROFILE_IDS[prof])
    for n in SIZES:
        note("utf16<->utf32 %s n=%d" % (prof, n))
        check_u16_to_u32(ctx, synth.utf16_buffer(prof, n, rng))
        check_u32_to_u16(ctx, synth.utf32_buffer(prof, n, rng))


@pytest.mark.parametrize("rate", [1e-4, 3e-2])
def test_utf16_utf32_injected_errors(ctx, rate):
    rng = synth.rng_for(91, int(rate * 1e6))
    for prof in ("emoji", "mixed4"):
        inj = synth.inject_utf16(prof, 200_000, rate, rng)
        note("utf16->utf32 inject %s rate=%g" % (prof, rate))
        r = check_u16_to_u32(ctx, inj.data)
        assert r.status == utfx.E_SURROGATE and r.count == inj.positions[0]
        units, pos = synth.inject_utf32(synth.utf32_buffer(prof, 100_000, rng), rate, rng)
        note("utf32->utf16 inject %s rate=%g" % (prof, rate))
        r = check_u32_to_u16(ctx, units)
        assert r.status in (utfx.E_SURROGATE, utfx.E_TOO_LARGE) and r.count == pos[0]


def test_utf16_surrogate_error_at_every_chunk_offset(ctx):
    rng = synth.rng_for(92)
    base = synth.utf16_buffer("emoji", 3000, rng)
    for kind in synth.UTF16_KINDS:
        for off in range(0, 40):
            w = base.copy()
            if off > 0:
                w[off - 1] = 0x41
            if off > 1 and 0xD800 <= w[off - 2] < 0xDC00:
                w[off - 2] = 0x40
            w[off] = synth.utf16_error_item(kind, rng)[0]
            w[off + 1] = 0x42
            if 0xDC00 <= w[off + 2] < 0xE000:
                w[off + 2] = 0x43
            note("utf16->utf32 %s off=%d" % (kind, off))
            assert check_u16_to_u32(ctx, w).count == off


def test_utf16_utf32_alphabets(ctx):
    from test_oracle_pins import ALPHA16, ALPHA32, _all_strings

    for L in (1, 2, 3):
        note("utf16->utf32 alphabet L=%d" % L)
        for s in _all_strings(ALPHA16, L).astype(np.uint16):
            check_u16_to_u32(ctx, s, guard=8)
        note("utf32->utf16 alphabet L=%d" % L)
        for s in _all_strings(ALPHA32, L).astype(np.uint32):
            check_u32_to_u16(ctx, s, guard=8)


@pytest.mark.parametrize("shift", [0, 1, 3, 6])
def test_utf16_utf32_misaligned_and_capacity(ctx, shift):
    rng = synth.rng_for(93, shift)
    words = synth.utf16_buffer("emoji", 10_007, rng)
    units = synth.utf32_buffer("mixed4", 10_007, rng)
    note("utf16<->utf32 shift=%d" % shift)
    check_u16_to_u32(ctx, words, in_shift=shift, out_shift=shift % 4)
    check_u32_to_u16(ctx, units, in_shift=shift % 4, out_shift=shift)
    need = O.utf16le_to_utf32le(words)[0].count
    for cap in (0, 1, need - 1, need):
        r = check_u16_to_u32(ctx, words, cap=cap, out_shift=shift % 4)
        assert r.status == (utfx.OK if cap >= need else utfx.E_OUTPUT_TOO_SMALL)
    need = O.utf32le_to_utf16le(units)[0].count
    for cap in (0, 1, need - 1, need):
        r = check_u32_to_u16(ctx, units, cap=cap, out_shift=shift)
        assert r.status == (utfx.OK if cap >= need else utfx.E_OUTPUT_TOO_SMALL)


def test_utf16_utf32_async_and_round_trip(ctx):
    import torch

    rng = synth.rng_for(94)
    words = synth.utf16_buffer("mixed4", 1_000_003, rng)
    s16, _ = dev_u16(words)
    o32 = torch.empty(words.size, dtype=torch.int32, device="cuda")
    back = torch.empty(2 * words.size, dtype=torch.int16, device="cuda")
    res = utfx.result_tensor(2)
    assert ctx.utf16le_to_utf32le_async(s16, o32, res[0:24]) == utfx.OK
    torch.cuda.synchronize()
    r = utfx.results_from_tensor(res)[0]
    assert tuple(r) == tuple(O.utf16le_to_utf32le(words)[0])
    assert ctx.utf32le_to_utf16le_async(o32[: r.written], back, res[24:48]) == utfx.OK
    torch.cuda.synchronize()
    r2 = utfx.results_from_tensor(res)[1]
    assert tuple(r2) == (utfx.OK, words.size, words.size)
    assert np.array_equal(back[: words.size].cpu().numpy().view(np.uint16), words)


def test_utf16_utf32_full_size(ctx):
    import torch

    full = 256 << 20
    words = synth.config_buffer("emoji", synth.DIR_16TO8, full, config=2)
    note("utf16->utf32 full size")
    assert check_u16_to_u32(ctx, words).status == utfx.OK
    torch.cuda.empty_cache()
    units = synth.utf32_buffer("mixed4", full // 4, synth.rng_for(95))
    note("utf32->utf16 full size")
    assert check_u32_to_u16(ctx, units).status == utfx.OK
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prof", ["emoji", "mixed4", "cjk"])
def test_utf16be_utf32(ctx, prof):
    """UTF-16BE <-> UTF-32LE: ragged sizes, injected unpaired surrogates (dense enough for
    the rescan), misaligned pointers and small outputs, big-endian words on the UTF-16
    side."""
    rng = synth.rng_for(96, synth.PROFILE_IDS[prof])
    for n in (1, 2, 17, 4097, 8193, 300_007):
        note("utf16be<->utf32 %s n=%d" % (prof, n))
        check_u16_to_u32(ctx, synth.utf16_buffer(prof, n, rng).byteswap(), be=True)
        check_u32_to_u16(ctx, synth.utf32_buffer(prof, n, rng), be=True)
    for rate in (1e-4, 3e-2):
        inj = synth.inject_utf16(prof, 100_000, rate, rng)
        note("utf16be->utf32 inject %s rate=%g" % (prof, rate))
        r = check_u16_to_u32(ctx, inj.data.byteswap(), be=True)
        assert r.status == utfx.E_SURROGATE and r.count == inj.positions[0]
    words = synth.utf16_buffer(prof, 10_007, rng).byteswap()
    units = synth.utf32_buffer(prof, 10_007, rng)
    check_u16_to_u32(ctx, words, in_shift=3, out_shift=1, be=True)
    check_u32_to_u16(ctx, units, in_shift=1, out_shift=3, be=True)
    need = O.utf32le_to_utf16be(units)[0].count
    assert check_u32_to_u16(ctx, units, cap=need - 1, be=True).status == utfx.E_OUTPUT_TOO_SMALL
