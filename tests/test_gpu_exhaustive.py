"""Exhaustive short strings on the GPU through the batched call: every string of up to
4 bytes over 26 bytes that sit on every class edge of Table 1 (475,254 strings), and
every string of up to 4 words over 12 words on every UTF-16 class edge (22,620
strings), each compared with the oracle: status, offset, output length and output."""
import numpy as np
import pytest

import oracle as O
import paper_2212_05098_amd as utfx
from gpu_helpers import note

pytestmark = pytest.mark.gpu

ALPHA8 = [0x00, 0x7F, 0x80, 0x8F, 0x90, 0x9F, 0xA0, 0xBF, 0xC0, 0xC1, 0xC2, 0xDF, 0xE0, 0xE1,
          0xEC, 0xED, 0xEE, 0xEF, 0xF0, 0xF1, 0xF3, 0xF4, 0xF5, 0xF7, 0xF8, 0xFF]
ALPHA16 = [0x0000, 0x007F, 0x0080, 0x07FF, 0x0800, 0xD7FF, 0xD800, 0xDBFF, 0xDC00, 0xDFFF,
           0xE000, 0xFFFF]


def _all_strings(alpha, L):
    idx = np.indices([len(alpha)] * L).reshape(L, -1).T
    return np.array(alpha)[idx]


def _run(ctx, arena, in_off, in_len, dirs, caps, out_off, out_size):
    import torch

    n = len(in_off)
    d_in = torch.from_numpy(arena).cuda()
    d_out = torch.zeros(out_size, dtype=torch.uint8, device="cuda")
    items = utfx.pack_items(in_off, in_len, out_off, caps, dirs)
    res = utfx.result_tensor(n)
    assert ctx.batch_run(d_in, d_out, items, n, int(np.sum(in_len)), res) == utfx.OK
    torch.cuda.synchronize()
    b = res.cpu().numpy().view(np.uint8)
    rec = b.view(np.dtype([("status", "<i4"), ("reserved", "<u4"), ("count", "<u8"), ("written", "<u8")]))
    return rec, d_out.cpu().numpy()


def test_exhaustive_utf8_class_alphabet():
    strs = [_all_strings(ALPHA8, L).astype(np.uint8) for L in range(1, 5)]
    arena = np.concatenate([s.ravel() for s in strs] + [np.zeros(64, np.uint8)])
    in_len = np.concatenate([np.full(s.shape[0], s.shape[1], np.uint64) for s in strs])
    in_off = np.concatenate([[0], np.cumsum(in_len)[:-1]]).astype(np.uint64)
    n = in_len.size
    out_off = (2 * in_off).astype(np.uint64)  # a slot of in_len words each
    note("exhaustive utf8: %d strings" % n)
    with utfx.Context() as ctx:
        rec, out = _run(ctx, arena, in_off, in_len, np.zeros(n, np.uint32), in_len, out_off,
                        int(2 * in_off[-1] + 2 * in_len[-1] + 64))
    bad = 0
    for i in range(n):
        a, L = int(in_off[i]), int(in_len[i])
        want, ref = O.utf8_to_utf16le(arena[a:a + L])
        got = (int(rec["status"][i]), int(rec["count"][i]), int(rec["written"][i]))
        if got != tuple(want) or not np.array_equal(
                out[2 * a:2 * a + 2 * want.written].view(np.uint16), ref[:want.written]):
            bad += 1
            assert bad < 5, (arena[a:a + L].tobytes().hex(), got, want)
    assert bad == 0


def test_exhaustive_utf16_class_alphabet():
    strs = [_all_strings(ALPHA16, L).astype(np.uint16) for L in range(1, 5)]
    words = np.concatenate([s.ravel() for s in strs] + [np.zeros(32, np.uint16)])
    arena = words.astype("<u2").view(np.uint8).copy()
    in_len = np.concatenate([np.full(s.shape[0], s.shape[1], np.uint64) for s in strs])
    in_off_w = np.concatenate([[0], np.cumsum(in_len)[:-1]]).astype(np.uint64)
    n = in_len.size
    caps = 3 * in_len
    out_off = (3 * in_off_w).astype(np.uint64)
    note("exhaustive utf16: %d strings" % n)
    with utfx.Context() as ctx:
        rec, out = _run(ctx, arena, 2 * in_off_w, in_len, np.ones(n, np.uint32), caps, out_off,
                        int(out_off[-1] + caps[-1] + 64))
    for i in range(n):
        a, L = int(in_off_w[i]), int(in_len[i])
        want, ref = O.utf16le_to_utf8(words[a:a + L])
        got = (int(rec["status"][i]), int(rec["count"][i]), int(rec["written"][i]))
        o = int(out_off[i])
        assert got == tuple(want), (words[a:a + L], got, want)
        assert np.array_equal(out[o:o + want.written], ref[:want.written])
