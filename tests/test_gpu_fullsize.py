"""Parity at the benchmark's full size and launch configuration: each 256 MiB buffer the
benchmark times (four script profiles, both directions, the tuned launch configuration
it loads) transcoded, validated and measured on the GPU, compared with the oracle
element by element over the whole output; then full-size buffers with errors injected at
rates of 1e-6 and 1e-3, and buffers truncated in their last character."""
import numpy as np
import pytest

import oracle as O
import paper_2212_05098_amd as utfx
from paper_2212_05098_amd import synth
from gpu_helpers import check_u16_to_u8, check_u8_to_u16, dev_u8, dev_u16, note

pytestmark = pytest.mark.gpu

FULL = 256 << 20


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available()
    c = utfx.Context()
    assert c.load_tuning(), "the tuning cache the benchmark loads is missing"
    yield c
    c.close()


@pytest.mark.parametrize("prof", synth.SCRIPT_PROFILES)
def test_full_size_utf8_to_utf16(ctx, prof):
    import torch

    data = synth.config_buffer(prof, synth.DIR_8TO16, FULL, config=2)
    note("full size utf8->utf16 %s tuning=%s" % (prof, ctx.get_tuning(utfx.OP_UTF8_TO_UTF16)))
    r = check_u8_to_u16(ctx, data)
    assert r.status == utfx.OK and r.count == r.written
    src, _ = dev_u8(data)
    assert tuple(ctx.validate_utf8(src)) == tuple(O.validate_utf8(data))
    assert tuple(ctx.utf16_length_from_utf8(src)) == tuple(O.utf16_length_from_utf8(data))
    del src
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prof", synth.SCRIPT_PROFILES)
def test_full_size_utf16_to_utf8(ctx, prof):
    import torch

    words = synth.config_buffer(prof, synth.DIR_16TO8, FULL, config=2)
    note("full size utf16->utf8 %s tuning=%s" % (prof, ctx.get_tuning(utfx.OP_UTF16_TO_UTF8)))
    r = check_u16_to_u8(ctx, words)
    assert r.status == utfx.OK and r.count == r.written
    src, _ = dev_u16(words)
    assert tuple(ctx.validate_utf16le(src)) == tuple(O.validate_utf16le(words))
    assert tuple(ctx.utf8_length_from_utf16le(src)) == tuple(O.utf8_length_from_utf16le(words))
    del src
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prof,rate", [("cjk", 1e-6), ("cjk", 1e-3), ("mixed4", 1e-6), ("mixed4", 1e-3)])
def test_full_size_injected_utf8(ctx, prof, rate):
    """256 MiB with errors of every kind injected at the given rate: the verdict and
    first-error offset of the transcode and of validation, and the valid prefix."""
    import torch

    rng = synth.rng_for(40, synth.PROFILE_IDS[prof], int(rate * 1e6))
    inj = synth.inject_utf8(prof, FULL, rate, rng)
    note("full size utf8 %s rate %g: %d errors, first at %d" % (prof, rate, len(inj.positions), inj.positions[0]))
    r = check_u8_to_u16(ctx, inj.data)
    assert r.status != utfx.OK and r.count == inj.positions[0]
    src, _ = dev_u8(inj.data)
    assert tuple(ctx.validate_utf8(src)) == tuple(O.validate_utf8(inj.data))
    del src
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prof,rate", [("cjk", 1e-6), ("cjk", 1e-3), ("mixed4", 1e-6), ("mixed4", 1e-3)])
def test_full_size_injected_utf16(ctx, prof, rate):
    import torch

    rng = synth.rng_for(42, synth.PROFILE_IDS[prof], int(rate * 1e6))
    inj = synth.inject_utf16(prof, FULL // 2, rate, rng)
    note("full size utf16 %s rate %g: %d errors, first at %d" % (prof, rate, len(inj.positions), inj.positions[0]))
    r = check_u16_to_u8(ctx, inj.data)
    assert r.status == utfx.E_SURROGATE and r.count == inj.positions[0]
    src, _ = dev_u16(inj.data)
    assert tuple(ctx.validate_utf16le(src)) == tuple(O.validate_utf16le(inj.data))
    del src
    torch.cuda.empty_cache()


def test_full_size_truncated_at_end(ctx):
    """A valid 256 MiB CJK buffer whose last character is cut short: the error sits at
    the very end, so the whole buffer before it is transcoded and compared."""
    import torch

    data = synth.config_buffer("cjk", synth.DIR_8TO16, FULL, config=2).copy()
    lead = data.size - 1
    while data[lead] & 0xC0 == 0x80:
        lead -= 1
    data[lead:] = 0x41
    data[-2:] = (0xE4, 0xB8)  # a 3-byte lead and one continuation, then the end
    note("full size utf8 truncated at the end")
    r = check_u8_to_u16(ctx, data)
    assert r.status == utfx.E_MISSING_CONT and r.count == data.size - 2
    words = synth.config_buffer("cjk", synth.DIR_16TO8, FULL, config=2).copy()
    words[-1] = 0xD83D  # a high surrogate with nothing after it
    r = check_u16_to_u8(ctx, words)
    assert r.status == utfx.E_SURROGATE and r.count == words.size - 1
    torch.cuda.empty_cache()
