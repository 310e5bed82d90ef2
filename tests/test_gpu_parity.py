"""GPU parity: the HIP library (through its C ABI) against the scalar CPU oracle on
the same seeded inputs.  Everything is integer, so the bar is bit-exact: status,
error offset, output length and every output unit of the valid prefix; nothing may
be stored at or beyond cap."""
import numpy as np
import pytest

import oracle as O
import paper_2212_05098_amd as utfx
from paper_2212_05098_amd import synth
from conftest import read_golden
from gpu_helpers import check_u16_to_u8, check_u8_to_u16, dev_u8, dev_u16, note

pytestmark = pytest.mark.gpu

# Launch configurations, (tile bytes, tiles per segment) per operation: small segments
# put many segment boundaries inside the test inputs, large ones exercise the
# per-tile scan inside a segment.  The transcodes take a fixed set of pairs (their
# segment lives in registers and its output in LDS); the other kernels take any.
TILES = (
    {"u8": (4096, 2), "u16": (4096, 2), "other": (4096, 1)},
    {"u8": (4096, 4), "u16": (4096, 8), "other": (8192, 3)},
    {"u8": (8192, 2), "u16": (8192, 4), "other": (8192, 8)},
    {"u8": (4096, 8), "u16": (8192, 8), "other": (4096, 32)},
    {"u8": (8192, 2), "u16": (4096, 2), "other": (8192, 4)},
)
OPS = (utfx.OP_UTF8_TO_UTF16, utfx.OP_UTF16_TO_UTF8, utfx.OP_VALIDATE_UTF8, utfx.OP_VALIDATE_UTF16,
       utfx.OP_LENGTH_UTF8, utfx.OP_LENGTH_UTF16)


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available()
    c = utfx.Context()
    yield c
    c.close()


def set_tile(ctx, T):
    """T: a TILES entry, or one (tile bytes, tiles per segment) pair for every op."""
    if isinstance(T, tuple):
        T = {"u8": T, "u16": T, "other": T}
    for op in OPS:
        key = {utfx.OP_UTF8_TO_UTF16: "u8", utfx.OP_UTF16_TO_UTF8: "u16"}.get(op, "other")
        ctx.set_tuning(op, *T[key])


def hx(s):
    return [int(t, 16) for t in s.split()]


def test_library_is_the_hip_build(ctx):
    import os

    assert os.path.samefile(utfx.lib()._name, utfx.LIBRARY)


def test_config1_round_trip(ctx):
    """64 KiB mixed buffer, seed 0: UTF-8 -> UTF-16LE and back, against the oracle."""
    import torch

    data = synth.config1_buffer()
    for T in TILES:
        note("config1 T=%s" % (T,))
        set_tile(ctx, T)
        r = check_u8_to_u16(ctx, data)
        assert r.status == utfx.OK
        words = O.utf8_to_utf16le(data)[1][: r.written]
        r2 = check_u16_to_u8(ctx, words)
        assert r2 == (utfx.OK, data.size, data.size)
    set_tile(ctx, TILES[1])


def test_golden_rules(ctx):
    for d, units, st, cnt in read_golden("rules.txt"):
        note("rules %s %s" % (d, units))
        if d == "u8":
            check_u8_to_u16(ctx, np.array(hx(units), dtype=np.uint8))
        else:
            check_u16_to_u8(ctx, np.array(hx(units), dtype=np.uint16))


def test_golden_paper_examples(ctx):
    for cp, u16, u8 in read_golden("fig1b_codepoints.txt"):
        note("fig1b %s" % cp)
        check_u8_to_u16(ctx, np.array(hx(u8), dtype=np.uint8))
        check_u16_to_u8(ctx, np.array(hx(u16), dtype=np.uint16))
    for label, u8, u16 in read_golden("worked_examples.txt"):
        note("example %s" % label)
        r = check_u8_to_u16(ctx, np.array(hx(u8), dtype=np.uint8))
        assert r.status == utfx.OK


def test_all_scalar_values(ctx):
    cps = np.concatenate([np.arange(0, 0xD800), np.arange(0xE000, 0x110000)]).astype(np.uint32)
    s = synth.cps_to_str(cps)
    u8 = np.frombuffer(s.encode("utf-8"), dtype=np.uint8)
    u16 = np.frombuffer(s.encode("utf-16-le"), dtype="<u2").astype(np.uint16)
    for T in TILES:
        note("all scalar values T=%s" % (T,))
        set_tile(ctx, T)
        assert check_u8_to_u16(ctx, u8).status == utfx.OK
        assert check_u16_to_u8(ctx, u16).status == utfx.OK
    set_tile(ctx, TILES[1])


@pytest.mark.parametrize("prof", synth.SCRIPT_PROFILES + ("mixed4",))
def test_profiles_ragged_sizes(ctx, prof):
    rng = synth.rng_for(11, synth.PROFILE_IDS[prof])
    for n in (1, 2, 3, 5, 15, 16, 17, 63, 64, 65, 1000, 4095, 4096, 4097, 8191, 8193, 40_000, 300_007):
        note("profile %s n=%d" % (prof, n))
        check_u8_to_u16(ctx, synth.utf8_buffer(prof, n, rng))
        check_u16_to_u8(ctx, synth.utf16_buffer(prof, n, rng))


@pytest.mark.parametrize("prof", synth.SCRIPT_PROFILES)
def test_run_structured_text(ctx, prof):
    """Run-structured text (same-script words), where whole waves fall into one content
    class, in several launch configurations."""
    rng = synth.rng_for(17, synth.PROFILE_IDS[prof])
    for T in (TILES[0], TILES[2]):
        set_tile(ctx, T)
        for n in (255, 65_537, 1_000_003):
            note("run-structured %s n=%d T=%s" % (prof, n, T))
            check_u8_to_u16(ctx, synth.run_utf8_buffer(prof, n, rng))
            check_u16_to_u8(ctx, synth.run_utf16_buffer(prof, n // 2 + 1, rng))
    set_tile(ctx, TILES[1])


@pytest.mark.parametrize("shift", list(range(0, 16)))
def test_misaligned_pointers(ctx, shift):
    rng = synth.rng_for(12, shift)
    data = synth.utf8_buffer("mixed4", 20_011, rng)
    words = synth.utf16_buffer("emoji", 10_007, rng)
    note("misaligned shift=%d" % shift)
    check_u8_to_u16(ctx, data, in_shift=shift, out_shift=shift % 8)
    check_u8_to_u16(ctx, data, in_shift=(shift * 7) % 16, out_shift=(shift * 3) % 8)
    check_u16_to_u8(ctx, words, in_shift=shift % 8, out_shift=shift)


@pytest.mark.parametrize("prof", ["cjk", "latin", "mixed4", "emoji"])
@pytest.mark.parametrize("rate", [1e-4, 3e-3, 3e-2])
def test_injected_errors(ctx, prof, rate):
    rng = synth.rng_for(13, synth.PROFILE_IDS[prof], int(rate * 1e6))
    for T in TILES:
        set_tile(ctx, T)
        note("inject %s rate=%g T=%s" % (prof, rate, T))
        inj = synth.inject_utf8(prof, 200_000, rate, rng)
        r = check_u8_to_u16(ctx, inj.data)
        assert r.status != utfx.OK and r.count == inj.positions[0]
        inj = synth.inject_utf16(prof, 100_000, rate, rng)
        r = check_u16_to_u8(ctx, inj.data)
        assert r.status == utfx.E_SURROGATE and r.count == inj.positions[0]
    set_tile(ctx, TILES[1])


@pytest.mark.parametrize("kind", synth.UTF8_KINDS)
def test_each_utf8_error_kind_at_every_chunk_offset(ctx, kind):
    """One error item placed at every offset 0..80 of a valid run (covering every
    position inside a 16-byte chunk and chunk/wave edges)."""
    rng = synth.rng_for(14, synth.UTF8_KINDS.index(kind))
    base = synth.utf8_buffer("mixed4", 4000, rng).tobytes()
    for off in range(0, 81):
        item = synth.utf8_error_item(kind, rng)
        prefix = base[:off].decode("utf-8", errors="ignore").encode("utf-8")
        prefix += b"a" * (off - len(prefix))
        data = np.frombuffer(prefix + item + b"z" + base[off:], dtype=np.uint8)
        note("kind %s off=%d" % (kind, off))
        r = check_u8_to_u16(ctx, data)
        assert r.count == off


def test_utf16_error_at_every_chunk_offset(ctx):
    rng = synth.rng_for(15)
    base = synth.utf16_buffer("emoji", 3000, rng)
    for kind in synth.UTF16_KINDS:
        for off in range(0, 40):
            w = base.copy()
            # make off a character boundary with a plain BMP word before it
            if off > 0:
                w[off - 1] = 0x41
            if off > 1 and 0xD800 <= w[off - 2] < 0xDC00:
                w[off - 2] = 0x40
            w[off] = synth.utf16_error_item(kind, rng)[0]
            w[off + 1] = 0x42
            if 0xDC00 <= w[off + 2] < 0xE000:
                w[off + 2] = 0x43
            note("u16 %s off=%d" % (kind, off))
            r = check_u16_to_u8(ctx, w)
            assert r.count == off


@pytest.mark.parametrize("T,seg", [(4096, 2), (4096, 8), (8192, 4), (8192, 2)])
def test_tile_edges(ctx, T, seg):
    rng = synth.rng_for(16, T, seg)
    set_tile(ctx, (T, seg))
    for direction in (synth.DIR_8TO16, synth.DIR_16TO8):
        for data, at in synth.tile_edge_cases([T, T * seg], 6 * T * seg + 100, rng, direction):
            note("tile edge T=%d dir=%d at=%s" % (T, direction, at))
            if direction == synth.DIR_8TO16:
                r = check_u8_to_u16(ctx, data)
            else:
                r = check_u16_to_u8(ctx, data)
            if at is None:
                assert r.status == utfx.OK
            else:
                assert r.status != utfx.OK and r.count == at
    # truncated sequences and unpaired highs at the very end of the buffer
    for L in (T - 1, T, T + 1, 2 * T - 2):
        for tail in (b"\xc3", b"\xe2\x82", b"\xf0\x9f\x98", b"\xf0"):
            d = np.frombuffer(b"a" * (L - len(tail)) + tail, dtype=np.uint8)
            note("end tail T=%d L=%d" % (T, L))
            r = check_u8_to_u16(ctx, d)
            assert r.status == utfx.E_MISSING_CONT and r.count == L - len(tail)
        w = np.full(L // 2, 0x41, dtype=np.uint16)
        w[-1] = 0xD83D
        r = check_u16_to_u8(ctx, w)
        assert r.count == L // 2 - 1
    set_tile(ctx, TILES[1])


def test_output_capacity(ctx):
    rng = synth.rng_for(17)
    data = synth.utf8_buffer("mixed4", 50_000, rng)
    need = O.utf16_length_from_utf8(data).count
    for cap in (0, 1, 7, 8, 9, need // 2, need - 1, need, need + 5):
        note("cap u8 %d" % cap)
        r = check_u8_to_u16(ctx, data, cap=cap, out_shift=3)
        assert r.status == (utfx.OK if cap >= need else utfx.E_OUTPUT_TOO_SMALL)
    words = synth.utf16_buffer("cjk", 20_000, rng)
    need = O.utf8_length_from_utf16le(words).count
    for cap in (0, 1, 15, 16, 17, need - 1, need):
        note("cap u16 %d" % cap)
        r = check_u16_to_u8(ctx, words, cap=cap, out_shift=5)
        assert r.status == (utfx.OK if cap >= need else utfx.E_OUTPUT_TOO_SMALL)
    # an error outranks a small buffer; the valid prefix still lands below cap
    inj = synth.inject_utf8("cjk", 50_000, 1e-4, rng)
    check_u8_to_u16(ctx, inj.data, cap=10)


def test_empty_and_arguments(ctx):
    import torch

    e = torch.zeros(0, dtype=torch.uint8, device="cuda")
    assert ctx.validate_utf8(e) == (utfx.OK, 0, 0)
    assert ctx.utf16_length_from_utf8(e) == (utfx.OK, 0, 0)
    o = torch.zeros(4, dtype=torch.int16, device="cuda")
    assert ctx.utf8_to_utf16le(e, o) == (utfx.OK, 0, 0)
    # misaligned UTF-16 pointer and null input are argument errors, nothing launched
    b = torch.zeros(64, dtype=torch.uint8, device="cuda")
    r = ctx.raw("utfx_validate_utf16le", b.data_ptr() + 1, 4)
    assert r.status == utfx.E_INVALID_ARG
    r = ctx.raw("utfx_validate_utf8", None, 4)
    assert r.status == utfx.E_INVALID_ARG
    r = ctx.raw("utfx_utf8_to_utf16le", b.data_ptr(), 4, None, 4)
    assert r.status == utfx.E_INVALID_ARG


def test_random_garbage(ctx):
    """Random and lightly corrupted bytes: most inputs fail early or at odd places."""
    rng = synth.rng_for(18)
    for i in range(60):
        n = int(rng.integers(1, 5000))
        if i % 2:
            data = rng.integers(0, 256, size=n, dtype=np.uint8)
        else:
            data = synth.utf8_buffer("mixed4", n, rng)
            flips = rng.integers(0, n, size=max(1, n // 500))
            data[flips] = rng.integers(0, 256, size=flips.size, dtype=np.uint8)
        note("garbage u8 i=%d n=%d" % (i, n))
        check_u8_to_u16(ctx, data)
        w = rng.choice(np.array([0x41, 0x7FF, 0x800, 0xD800, 0xDBFF, 0xDC00, 0xDFFF, 0xFFFF], np.uint16),
                       size=max(1, n // 2))
        note("garbage u16 i=%d n=%d" % (i, n))
        check_u16_to_u8(ctx, w)


def test_class_alphabet_short_strings(ctx):
    """Every string of length <= 3 over the 26 class-edge bytes, and length <= 3 over
    the 12 class-edge words, through the single-buffer calls."""
    from test_oracle_pins import ALPHA8, ALPHA16, _all_strings

    for L in (1, 2, 3):
        strs = _all_strings(ALPHA8, L).astype(np.uint8)
        note("alphabet u8 L=%d (%d strings)" % (L, strs.shape[0]))
        for s in strs:
            check_u8_to_u16(ctx, s, guard=8)
        strs = _all_strings(ALPHA16, L).astype(np.uint16)
        note("alphabet u16 L=%d" % L)
        for s in strs:
            check_u16_to_u8(ctx, s, guard=8)


def test_async_result_buffer(ctx):
    import torch

    data = synth.config1_buffer()
    src, _ = dev_u8(data)
    dst = torch.empty(data.size, dtype=torch.int16, device="cuda")
    res = utfx.result_tensor(3)
    assert ctx.utf8_to_utf16le_async(src, dst, res[0:24]) == utfx.OK
    assert ctx.validate_utf8_async(src, res[24:48]) == utfx.OK
    assert ctx.utf16_length_from_utf8_async(src, res[48:72]) == utfx.OK
    torch.cuda.synchronize()
    r = utfx.results_from_tensor(res)
    want = O.utf8_to_utf16le(data)[0]
    assert tuple(r[0]) == tuple(want)
    assert tuple(r[1]) == tuple(O.validate_utf8(data))
    assert tuple(r[2]) == tuple(O.utf16_length_from_utf8(data))


@pytest.mark.parametrize("wgs", [1, 2, 3, 4])
def test_residency_cap_same_results(wgs):
    """Capping the resident workgroups per CU (utfx_set_tuning's wgs_per_cu, through
    unused dynamic LDS) changes the schedule, never the results: both transcodes,
    validation and the length queries on 8 MiB buffers with an error late in one."""
    rng = synth.rng_for(12, wgs)
    d8 = synth.utf8_buffer("mixed4", (8 << 20) + 5, rng)
    bad = d8.copy()
    bad[bad.size - 3000] = 0xC1
    w = synth.utf16_buffer("emoji", (4 << 20) + 3, rng)
    with utfx.Context() as c:
        for op in range(6):
            t, s_, _ = c.get_tuning(op)
            c.set_tuning(op, t, s_, wgs)
        note("residency cap %d" % wgs)
        for data in (d8, bad):
            check_u8_to_u16(c, data)
            src, _ = dev_u8(data)
            assert tuple(c.validate_utf8(src)) == tuple(O.validate_utf8(data))
            assert tuple(c.utf16_length_from_utf8(src)) == tuple(O.utf16_length_from_utf8(data))
        check_u16_to_u8(c, w)
        src, _ = dev_u16(w)
        assert tuple(c.validate_utf16le(src)) == tuple(O.validate_utf16le(w))
        assert tuple(c.utf8_length_from_utf16le(src)) == tuple(O.utf8_length_from_utf16le(w))
