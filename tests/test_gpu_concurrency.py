"""Contexts on different streams run at the same time without interfering: each owns
its workspace (status words, error word, epoch), so two transcodes in flight at once,
one of them on invalid input, both match the oracle; repeated back-to-back calls on one
context (epochs advancing without any clearing) stay exact."""
import numpy as np
import pytest

import oracle as O
import paper_2212_05098_amd as utfx
from paper_2212_05098_amd import synth
from gpu_helpers import note

pytestmark = pytest.mark.gpu


def _u8_case(prof, n, rng, bad_at=None):
    data = synth.utf8_buffer(prof, n, rng)
    if bad_at is not None:
        data[bad_at] = 0xC0
    return data


def test_two_streams_in_flight():
    import torch

    rng = synth.rng_for(50, 1)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    c1, c2 = utfx.Context(s1), utfx.Context(s2)
    try:
        a = _u8_case("cjk", 24 << 20, rng)
        b = _u8_case("emoji", 24 << 20, rng, bad_at=(17 << 20) + 5)
        words = synth.utf16_buffer("latin", 12 << 20, rng)
        da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        dw = torch.from_numpy(words.view(np.int16)).cuda()
        oa = torch.empty(a.size, dtype=torch.int16, device="cuda")
        ob = torch.empty(b.size, dtype=torch.int16, device="cuda")
        ow = torch.empty(3 * words.size, dtype=torch.uint8, device="cuda")
        res = utfx.result_tensor(3)
        torch.cuda.synchronize()
        note("two streams: utf8 cjk on s1, utf8 emoji (invalid) and utf16 on s2")
        for _ in range(3):
            with torch.cuda.stream(s1):
                assert c1.utf8_to_utf16le_async(da, oa, res[0:24]) == utfx.OK
            with torch.cuda.stream(s2):
                assert c2.utf8_to_utf16le_async(db, ob, res[24:48]) == utfx.OK
                assert c2.utf16le_to_utf8_async(dw, ow, res[48:72]) == utfx.OK
            torch.cuda.synchronize()
            got = utfx.results_from_tensor(res)
            for (data, out, r, fn) in ((a, oa, got[0], O.utf8_to_utf16le), (b, ob, got[1], O.utf8_to_utf16le),
                                       (words, ow, got[2], O.utf16le_to_utf8)):
                want, ref = fn(data)
                assert tuple(r) == tuple(want)
                host = out.cpu().numpy()
                host = host.view(np.uint16) if host.dtype == np.int16 else host
                assert np.array_equal(host[: want.written], ref[: want.written])
    finally:
        c1.close()
        c2.close()


def test_many_calls_one_context():
    """200 small calls in a row on one context, valid and invalid alternating, each
    result checked: the per-call epoch and error word never leak between calls."""
    import torch

    rng = synth.rng_for(50, 2)
    with utfx.Context() as ctx:
        for i in range(200):
            n = int(rng.integers(1, 70_000))
            bad = int(rng.integers(0, n)) if i % 2 else None
            data = _u8_case("mixed4", n, rng, bad_at=bad)
            src = torch.from_numpy(data).cuda()
            out = torch.empty(max(n, 1), dtype=torch.int16, device="cuda")
            r = ctx.utf8_to_utf16le(src, out)
            want, ref = O.utf8_to_utf16le(data)
            assert tuple(r) == tuple(want), (i, n, bad)
            v = ctx.validate_utf8(src)
            assert tuple(v) == tuple(O.validate_utf8(data)), (i, n, bad)
