"""Streams through the C ABI: a buffer cut into chunks at arbitrary unit offsets and
passed chunk by chunk must give what the oracle gives for the whole buffer: the same
output (the calls' outputs laid end to end), the same verdict and the same first-error
offset in stream coordinates.  After every successful call the stream has transcoded
exactly the complete characters so far: the oracle on that prefix of the concatenation
is OK and equals the output so far, and at most one unfinished character (3 bytes, or
one high surrogate) is carried."""
import numpy as np
import pytest

import oracle as O
import paper_2212_05098_amd as utfx
from paper_2212_05098_amd import synth
from gpu_helpers import note

pytestmark = pytest.mark.gpu

FORMATS = {
    utfx.STREAM_UTF8_TO_UTF16LE: (False, O.utf8_to_utf16le),
    utfx.STREAM_UTF16LE_TO_UTF8: (True, O.utf16le_to_utf8),
    utfx.STREAM_UTF8_TO_UTF16BE: (False, O.utf8_to_utf16be),
    utfx.STREAM_UTF16BE_TO_UTF8: (True, O.utf16be_to_utf8),
}
FILL8, FILL16 = 0xA5, 0x5A5A


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available()
    c = utfx.Context()
    yield c
    c.close()


def _dev(data, in16):
    import torch

    if in16:
        return torch.from_numpy(np.array(data, dtype=np.uint16).view(np.int16)).cuda()
    return torch.from_numpy(np.array(data, dtype=np.uint8)).cuda()


def run_stream(ctx, fmt, data, cuts, check_prefixes=True):
    """Pass data[cuts[i]:cuts[i+1]] call by call (the last one final); compare with the
    oracle on the whole buffer.  Returns the list of per-call results."""
    import torch

    in16, ref_fn = FORMATS[fmt]
    data = np.ascontiguousarray(data, dtype=np.uint16 if in16 else np.uint8)
    n = data.size
    src = _dev(data, in16)
    ocap = 3 * n + 8 if in16 else n + 8
    out = (torch.full((ocap + 64,), FILL8, dtype=torch.uint8, device="cuda") if in16 else
           torch.full((ocap + 64,), FILL16, dtype=torch.int16, device="cuda"))
    st = ctx.open_stream(fmt)
    want, ref = ref_fn(data)
    pos, results, err = 0, [], None
    for i in range(len(cuts) - 1):
        a, b = cuts[i], cuts[i + 1]
        final = i == len(cuts) - 2
        room = (st.n_carry + (b - a)) * (3 if in16 else 1)
        r = st.transcode(src[a:b], out[pos:pos + room], final=final)
        results.append(r)
        if err is not None:
            assert tuple(r) == (err.status, err.count, 0), (i, r, err)
            continue
        if r.status != utfx.OK:
            assert r.status == want.status and r.count == want.count, (i, r, want)
            assert pos + r.written == want.written, (i, pos, r, want)
            err = r
            continue
        pos += r.written
        assert st.out_units == pos and st.in_units == b
        done = b - st.n_carry  # stream offset of the first unit not yet transcoded
        assert st.n_carry <= (1 if in16 else 3) and done <= b
        if check_prefixes and (i % 7 == 0 or final):
            pw, pref = ref_fn(data[:done])
            assert pw.status == utfx.OK and pw.count == pos, (i, done, pw, pos)
            got = out[:pos].cpu().numpy()
            got = got.view(np.uint16) if got.dtype == np.int16 else got
            assert np.array_equal(got, pref[:pos]), i
    if err is None:
        assert want.status == utfx.OK and pos == want.written and st.n_carry == 0, (want, pos)
        got = out.cpu().numpy()
        got = got.view(np.uint16) if got.dtype == np.int16 else got
        assert np.array_equal(got[:pos], ref[:pos])
        assert np.all(got[pos:] == (FILL8 if in16 else FILL16)), "stored beyond the output"
    else:
        got = out[:want.written].cpu().numpy()
        got = got.view(np.uint16) if got.dtype == np.int16 else got
        assert np.array_equal(got, ref[:want.written])
    return results


def _buffer(fmt, prof, n, rng):
    in16, _ = FORMATS[fmt]
    if not in16:
        return synth.utf8_buffer(prof, n, rng)
    w = synth.utf16_buffer(prof, n, rng)
    return w.byteswap() if fmt == utfx.STREAM_UTF16BE_TO_UTF8 else w


@pytest.mark.parametrize("fmt", list(FORMATS))
@pytest.mark.parametrize("prof", ["mixed4", "emoji", "cjk", "latin"])
def test_valid_streams_random_cuts(ctx, fmt, prof):
    rng = synth.rng_for(70, fmt, synth.PROFILE_IDS[prof])
    for n, max_chunk in ((300, 1), (2_000, 9), (60_000, 5_000), (1_000_003, 200_000)):
        data = _buffer(fmt, prof, n, rng)
        cuts = synth.stream_cuts(data.size, rng, max_chunk)
        note("stream fmt=%d %s n=%d chunks=%d" % (fmt, prof, n, len(cuts) - 1))
        run_stream(ctx, fmt, data, cuts)


@pytest.mark.parametrize("fmt", list(FORMATS))
def test_every_two_chunk_split(ctx, fmt):
    """One short buffer (every UTF-8 length, a surrogate pair, an error near the end in
    half of the cases) split into two chunks at every offset."""
    in16, _ = FORMATS[fmt]
    if in16:
        base = [0x41, 0xE9, 0x4E2D, 0xD83D, 0xDE00, 0x20AC, 0xD800, 0xDC00, 0x7A]
        bad = base[:5] + [0xDC00] + base[5:]
        cases = [np.array(base, np.uint16), np.array(bad, np.uint16)]
        if fmt == utfx.STREAM_UTF16BE_TO_UTF8:
            cases = [c.byteswap() for c in cases]
    else:
        s = "aé中😀€\U00010000z".encode("utf-8")
        cases = [np.frombuffer(s, np.uint8), np.frombuffer(s[:5] + b"\xe2\x82" + s[5:], np.uint8),
                 np.frombuffer(s + b"\xf0\x9f", np.uint8), np.frombuffer(b"\xed\xa0\x80" + s, np.uint8)]
    for ci, data in enumerate(cases):
        for k in range(data.size + 1):
            note("two-chunk fmt=%d case=%d k=%d" % (fmt, ci, k))
            run_stream(ctx, fmt, data, [0, k, data.size])
        note("one unit per chunk fmt=%d case=%d" % (fmt, ci))
        run_stream(ctx, fmt, data, list(range(data.size + 1)))


@pytest.mark.parametrize("fmt", [utfx.STREAM_UTF8_TO_UTF16LE, utfx.STREAM_UTF16LE_TO_UTF8])
def test_injected_errors(ctx, fmt):
    in16, _ = FORMATS[fmt]
    for rate in (1e-5, 1e-3):
        rng = synth.rng_for(71, fmt, int(rate * 1e6))
        for trial in range(4):
            inj = (synth.inject_utf16("emoji", 200_000, rate, rng) if in16 else
                   synth.inject_utf8("mixed4", 400_000, rate, rng))
            cuts = synth.stream_cuts(inj.data.size, rng, 30_000)
            note("stream inject fmt=%d rate=%g trial=%d first=%d" % (fmt, rate, trial, inj.positions[0]))
            rs = run_stream(ctx, fmt, inj.data, cuts, check_prefixes=False)
            assert any(r.status not in (utfx.OK,) for r in rs)


def test_error_kinds_across_cuts(ctx):
    """Each UTF-8 error kind placed so that its character straddles a cut, at every
    offset of the cut within the bad item."""
    rng = synth.rng_for(72)
    head = synth.utf8_buffer("cjk", 1000, rng).tobytes()
    for kind in synth.UTF8_KINDS:
        item = synth.utf8_error_item(kind, rng)
        data = np.frombuffer(head + item + b"tail", np.uint8)
        for k in range(len(head) - 4, len(head) + len(item) + 2):
            note("kind %s cut at %d" % (kind, k))
            run_stream(ctx, utfx.STREAM_UTF8_TO_UTF16LE, data, [0, k, data.size])


def test_output_too_small_then_retry(ctx):
    import torch

    rng = synth.rng_for(73)
    data = synth.utf8_buffer("emoji", 10_000, rng)
    src = _dev(data, False)
    st = ctx.open_stream(utfx.STREAM_UTF8_TO_UTF16LE)
    out = torch.empty(20_000, dtype=torch.int16, device="cuda")
    r = st.transcode(src[:4001], out[:4001])
    assert r.status == utfx.OK
    pos, done = r.written, st.in_units
    saved = (st.in_units, st.out_units, st.n_carry, bytes(st.state.carry), st.state.carry_need)
    small = st.transcode(src[4001:], out[pos:pos + 10], final=True)
    assert small.status == utfx.E_OUTPUT_TOO_SMALL and small.written == 0
    assert (st.in_units, st.out_units, st.n_carry, bytes(st.state.carry), st.state.carry_need) == saved
    want, ref = O.utf8_to_utf16le(data)
    assert small.count == want.written - pos
    r = st.transcode(src[4001:], out[pos:pos + small.count], final=True)
    assert r == (utfx.OK, small.count, small.count)
    assert np.array_equal(out[: want.written].cpu().numpy().view(np.uint16), ref[: want.written])
    assert done == 4001


def test_state_rules(ctx):
    import torch

    st = ctx.open_stream(utfx.STREAM_UTF8_TO_UTF16LE)
    src = _dev(np.frombuffer("ab€".encode("utf-8"), np.uint8), False)
    out = torch.zeros(16, dtype=torch.int16, device="cuda")
    e = torch.zeros(0, dtype=torch.uint8, device="cuda")
    assert st.transcode(src[:3], out) == (utfx.OK, 2, 2) and st.n_carry == 1
    assert st.transcode(e, out) == (utfx.OK, 0, 0) and st.n_carry == 1   # empty chunk: carry kept
    r = st.transcode(src[3:4], out, final=True)  # still one byte short at the end
    assert r.status == utfx.E_MISSING_CONT and r.count == 2 and r.written == 0
    assert st.transcode(src, out) == (utfx.E_MISSING_CONT, 2, 0)         # the stream is over
    st2 = ctx.open_stream(utfx.STREAM_UTF8_TO_UTF16LE)
    assert st2.transcode(src, out, final=True) == (utfx.OK, 3, 3)
    assert st2.transcode(e, out).status == utfx.E_INVALID_ARG              # after the final chunk
    st3 = ctx.open_stream(utfx.STREAM_UTF16LE_TO_UTF8)
    b = torch.zeros(8, dtype=torch.uint8, device="cuda")
    assert st3.raw(b.data_ptr() + 1, 2, b.data_ptr(), 8).status == utfx.E_INVALID_ARG  # odd UTF-16 address
    assert st3.state.in_units == 0
    w = _dev(np.array([0x41, 0xD83D], np.uint16), True)
    assert st3.transcode(w, b) == (utfx.OK, 1, 1) and st3.n_carry == 1
    assert st3.transcode(e.view(torch.int16), b, final=True) == (utfx.E_SURROGATE, 1, 0)


def test_misaligned_chunks(ctx):
    rng = synth.rng_for(74)
    data = synth.utf8_buffer("mixed4", 50_000, rng)
    cuts = synth.stream_cuts(data.size, rng, 3_001, min_chunk=1)  # every chunk starts at a new byte offset
    note("stream misaligned chunks")
    run_stream(ctx, utfx.STREAM_UTF8_TO_UTF16BE, data, cuts)


def test_full_size_stream(ctx):
    """256 MiB of mixed text in chunks of up to 24 MiB cut at arbitrary byte offsets,
    in the tuned launch configuration the benchmark uses."""
    import torch

    assert ctx.load_tuning()
    rng = synth.rng_for(75)
    data = synth.config_buffer("mixed4", synth.DIR_8TO16, 256 << 20, config=2)
    cuts = synth.stream_cuts(data.size, rng, 24 << 20, min_chunk=1 << 20)
    note("stream 256 MiB in %d chunks" % (len(cuts) - 1))
    run_stream(ctx, utfx.STREAM_UTF8_TO_UTF16LE, data, cuts, check_prefixes=False)
    torch.cuda.empty_cache()
