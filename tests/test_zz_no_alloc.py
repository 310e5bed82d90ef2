"""The allocation-free UTF-8 -> UTF-16LE call (utfx_utf8_to_utf16le_noalloc, through the
C ABI) against the context call it is a variant of (utfx_utf8_to_utf16le_async) and the
oracle: two calls in a row on the shared static workspace, the second smaller, with
valid input, an injected error and an undersized output; then the size limit."""
import ctypes

import numpy as np
import pytest

import oracle as O
import paper_2212_05098_amd as utfx
from paper_2212_05098_amd import synth
from gpu_helpers import note

pytestmark = pytest.mark.gpu

GUARD = 0x5A5A


def _call_pair(ctx, data, cap, shift):
    """Runs the no-alloc call and the context call on the same bytes (input shifted by
    `shift` bytes from a 16-byte boundary); returns both results and outputs."""
    import torch

    n = data.size
    back = torch.zeros(n + shift + 16, dtype=torch.uint8, device="cuda")
    back[shift:shift + n] = torch.from_numpy(data.copy()).cuda()
    src = back[shift:shift + n]
    outs, results = [], []
    for which in ("noalloc", "ctx"):
        dst_back = torch.full((cap + 64,), GUARD, dtype=torch.int16, device="cuda")
        dst = dst_back[:cap]
        res = utfx.result_tensor(1)
        note("no-alloc %s: %d bytes, cap %d, shift %d" % (which, n, cap, shift))
        if which == "noalloc":
            st = utfx.utf8_to_utf16le_noalloc(src, dst, res)
        else:
            st = ctx.utf8_to_utf16le_async(src, dst, res)
        assert st == utfx.OK
        torch.cuda.synchronize()
        results.append(utfx.results_from_tensor(res)[0])
        outs.append(dst_back.cpu().numpy().view(np.uint16))
    return results, outs


def _check(ctx, data, cap, shift):
    (r_na, r_ctx), (o_na, o_ctx) = _call_pair(ctx, data, cap, shift)
    want, ref = O.utf8_to_utf16le(data, cap)
    assert tuple(r_na) == tuple(r_ctx) == tuple(want), (r_na, r_ctx, want)
    w = min(int(want.written), cap)
    assert np.array_equal(o_na[:w], ref[:w])
    assert np.array_equal(o_na[:w], o_ctx[:w])
    assert np.all(o_na[cap:] == GUARD)


def test_noalloc_matches_context_call_twice_then_smaller():
    import torch

    assert torch.cuda.is_available()
    rng = synth.rng_for(60, 1)
    big = synth.utf8_buffer("mixed4", (8 << 20) + 13, rng)
    small = synth.utf8_buffer("cjk", 70_001, rng)
    with utfx.Context() as ctx:
        # valid input, the second call smaller than the first
        _check(ctx, big, big.size, 0)
        _check(ctx, small, small.size, 5)
        # an error late in the big buffer, then an error early in the small one
        bad = big.copy()
        bad[big.size - 40_000] = 0xC0
        _check(ctx, bad, bad.size, 3)
        bad2 = small.copy()
        bad2[1234] = 0x80 if (bad2[1234] & 0xC0) != 0x80 else 0xFF
        _check(ctx, bad2, bad2.size, 0)
        # output too small
        want = O.utf16_length_from_utf8(small)
        _check(ctx, small, int(want.count) - 1, 1)
        # empty input
        res = utfx.result_tensor(1)
        assert utfx.utf8_to_utf16le_noalloc(torch.empty(0, dtype=torch.uint8, device="cuda"),
                                            torch.empty(0, dtype=torch.int16, device="cuda"), res) == utfx.OK
        torch.cuda.synchronize()
        assert tuple(utfx.results_from_tensor(res)[0]) == (utfx.OK, 0, 0)


def test_noalloc_rejects_sizes_and_pointers():
    """Rejected on the host with nothing queued: sizes above the limit, null pointers,
    a misaligned output (raw C ABI, so no tensor of that size is needed)."""
    import torch

    L = utfx.lib()
    res = utfx.result_tensor(1)
    buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
    p, r = buf.data_ptr(), res.data_ptr()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.utfx_utf8_to_utf16le_noalloc(p, utfx.NOALLOC_MAX_BYTES + 1, p, 16, r, stream) == utfx.E_INVALID_ARG
    assert L.utfx_utf8_to_utf16le_noalloc(None, 16, p, 16, r, stream) == utfx.E_INVALID_ARG
    assert L.utfx_utf8_to_utf16le_noalloc(p, 16, None, 16, r, stream) == utfx.E_INVALID_ARG
    assert L.utfx_utf8_to_utf16le_noalloc(p, 16, p, 16, None, stream) == utfx.E_INVALID_ARG
    assert L.utfx_utf8_to_utf16le_noalloc(p, 16, p + 1, 16, r, stream) == utfx.E_INVALID_ARG
    torch.cuda.synchronize()
