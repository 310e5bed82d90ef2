"""Look-back under delay injection: with UTFX_DEBUG_LOOKBACK_DELAY set when a context is
created, one segment in sixteen holds back its look-back publication for up to a few
ms, so waiting workgroups run out of patience and recompute their late predecessors'
aggregates from the input.  Every result must still match the oracle bit for bit:
single-buffer transcodes in both directions (with and without an error), a UTF-32
transcode, and a batch with long strings (segmented look-back, plan look-back)."""
import os

import numpy as np
import pytest

import oracle as O
import paper_2212_05098_amd as utfx
from paper_2212_05098_amd import synth
from gpu_helpers import compare_batch, note

pytestmark = pytest.mark.gpu

GUARD = 0xA5


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available()
    os.environ["UTFX_DEBUG_LOOKBACK_DELAY"] = "8"
    try:
        c = utfx.Context()
    finally:
        del os.environ["UTFX_DEBUG_LOOKBACK_DELAY"]
    yield c
    c.close()


@pytest.mark.parametrize("err_at", [None, 0.97])
def test_single_buffer_both_directions(ctx, err_at):
    import torch

    rng = synth.rng_for(70, 1 if err_at is None else 2)
    n = 64 << 20
    d8 = synth.utf8_buffer("mixed4", n, rng)
    if err_at is not None:
        d8[int(err_at * n)] = 0xFF
    note("delay-injected utf8->utf16le, %d bytes, error %s" % (n, err_at))
    src = torch.from_numpy(d8).cuda()
    dst = torch.full((n + 64,), 0x5A5A, dtype=torch.int16, device="cuda")
    r = ctx.utf8_to_utf16le(src, dst[:n])
    want, ref = O.utf8_to_utf16le(d8)
    assert tuple(r) == tuple(want)
    got = dst.cpu().numpy().view(np.uint16)
    assert np.array_equal(got[:want.written], ref[:want.written])
    assert np.all(got[n:] == 0x5A5A)

    w = synth.utf16_buffer("emoji", n // 2, rng)
    if err_at is not None:
        w[int(err_at * w.size)] = 0xDC00
    note("delay-injected utf16le->utf8, %d words" % w.size)
    src16 = torch.from_numpy(w.view(np.int16)).cuda()
    dst8 = torch.full((3 * w.size + 64,), GUARD, dtype=torch.uint8, device="cuda")
    r = ctx.utf16le_to_utf8(src16, dst8[:3 * w.size])
    want, ref = O.utf16le_to_utf8(w)
    assert tuple(r) == tuple(want)
    got = dst8.cpu().numpy()
    assert np.array_equal(got[:want.written], ref[:want.written])
    assert np.all(got[3 * w.size:] == GUARD)


def test_utf32(ctx):
    import torch

    rng = synth.rng_for(70, 3)
    n = 32 << 20
    d8 = synth.utf8_buffer("mixed4", n, rng)
    note("delay-injected utf8->utf32le, %d bytes" % n)
    src = torch.from_numpy(d8).cuda()
    dst = torch.empty(n, dtype=torch.int32, device="cuda")
    r = ctx.utf8_to_utf32le(src, dst)
    want, ref = O.utf8_to_utf32le(d8)
    assert tuple(r) == tuple(want)
    assert np.array_equal(dst.cpu().numpy().view(np.uint32)[:want.written], ref[:want.written])


def test_batch_with_long_strings(ctx):
    import torch

    b = synth.make_batch(20_000, seed_key=(70, 4), median=2048, sigma=2.0, hi=8 << 20, err_frac=0.01)
    caps, out_off, out_bytes = synth.batch_output_layout(b)
    items = O.items_array(b.in_off, b.in_len, out_off, caps, b.direction)
    ora_res, ora_out, _ = O.batch(b.arena, items, out_bytes)
    d_in = torch.from_numpy(b.arena).cuda()
    d_out = torch.full((out_bytes,), GUARD, dtype=torch.uint8, device="cuda")
    d_items = torch.from_numpy(items.view(np.uint8).copy()).cuda()
    res = utfx.result_tensor(len(b.in_len))
    note("delay-injected batch: %d strings, longest %d units" % (len(b.in_len), int(b.in_len.max())))
    assert ctx.batch_run(d_in, d_out, d_items, len(b.in_len), int(np.sum(b.in_len)), res) == utfx.OK
    torch.cuda.synchronize()
    compare_batch(res.cpu().numpy(), d_out.cpu().numpy(), ora_res, ora_out, items, "delay-injected", guard=GUARD)
