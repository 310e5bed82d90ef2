"""Exhaustive enumerations on the GPU, through the batched call (C ABI), against the
oracle item by item:

* every byte string of length <= 3 (16,843,008 strings) and every single UTF-16 word,
  the strings at every byte phase of the 16-byte chunk grid;
* every string of up to 5 bytes over the 26 class-edge bytes of Table 1 (12,356,630)
  and of up to 5 words over the 12 UTF-16 class-edge words, at varied phases; the
  strings of up to 3 class-edge bytes also through the single-buffer calls, one call
  each, at every phase;
* all 2^32 four-byte strings (UTF-8 -> UTF-16LE) and all 2^32 two-word strings
  (UTF-16LE -> UTF-8), in slices of 2^24 strings generated on the device: per-string
  status, offset and output length against the oracle, and the number of valid
  strings against the closed forms V(4) = 383,270,912 (section 2.2, Table 1) and
  U(2) = 63,488^2 + 1,024^2 = 4,031,774,720 (section 2.1).  About 20-40 s each on
  one MI355X and a 16-core host share, most of it the oracle.
"""
import concurrent.futures as cf
import os

import numpy as np
import pytest

import oracle as O
import paper_2212_05098_amd as utfx
from gpu_helpers import compare_batch, note

pytestmark = pytest.mark.gpu

ALPHA8 = [0x00, 0x7F, 0x80, 0x8F, 0x90, 0x9F, 0xA0, 0xBF, 0xC0, 0xC1, 0xC2, 0xDF, 0xE0, 0xE1,
          0xEC, 0xED, 0xEE, 0xEF, 0xF0, 0xF1, 0xF3, 0xF4, 0xF5, 0xF7, 0xF8, 0xFF]
ALPHA16 = [0x0000, 0x007F, 0x0080, 0x07FF, 0x0800, 0xD7FF, 0xD800, 0xDBFF, 0xDC00, 0xDFFF,
           0xE000, 0xFFFF]
GUARD = 0xA5


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available()
    c = utfx.Context()
    yield c
    c.close()


def _workers():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _layout(groups, unit):
    """Arena of groups of equal-length strings (rows of an array each).  A group of
    length L sits back to back, so odd L sweeps every phase of the 16-byte grid; even
    L is split in halves one unit apart.  Returns (arena bytes, in_off, in_len)."""
    parts, in_off, in_len = [], [], []
    off = 0
    for g in groups:
        n, L = g.shape
        halves = (g[: n // 2], g[n // 2:]) if L % 2 == 0 else (g,)
        for h in halves:
            raw = np.ascontiguousarray(h).astype("<u2" if unit == 2 else np.uint8).view(np.uint8).ravel()
            parts.append(raw)
            in_off.append(off + np.arange(h.shape[0], dtype=np.uint64) * (L * unit))
            in_len.append(np.full(h.shape[0], L, dtype=np.uint64))
            off += raw.size
            parts.append(np.zeros(unit, np.uint8))  # shifts the next half by one unit
            off += unit
    parts.append(np.zeros(64, np.uint8))
    return np.concatenate(parts), np.concatenate(in_off), np.concatenate(in_len)


def _run_batch(ctx, arena, in_off, in_len, direction, label):
    import torch

    n = in_off.size
    caps = (in_len if direction == 0 else 3 * in_len).astype(np.uint64)
    unit_out = 2 if direction == 0 else 1
    out_off = np.concatenate([[0], np.cumsum(caps * unit_out + 2)[:-1]]).astype(np.uint64)
    out_bytes = int(out_off[-1] + caps[-1] * unit_out + 64)
    dirs = np.full(n, direction, dtype=np.uint32)
    items = O.items_array(in_off, in_len, out_off, caps, dirs)
    ora_res, ora_out, n_ok = O.batch(arena, items, out_bytes)
    d_in = torch.from_numpy(arena).cuda()
    d_out = torch.full((out_bytes,), GUARD, dtype=torch.uint8, device="cuda")
    d_items = torch.from_numpy(items.view(np.uint8).copy()).cuda()
    res = utfx.result_tensor(n)
    note("%s: %d strings" % (label, n))
    assert ctx.batch_run(d_in, d_out, d_items, n, int(np.sum(in_len)), res) == utfx.OK, ctx.last_error()
    torch.cuda.synchronize()
    compare_batch(res.cpu().numpy(), d_out.cpu().numpy(), ora_res, ora_out, items, label, guard=GUARD)
    return n_ok


def _all_strings(alpha, L):
    idx = np.indices([len(alpha)] * L).reshape(L, -1).T
    return np.array(alpha)[idx]


def test_every_string_up_to_3_bytes_at_every_phase(ctx):
    groups = []
    for L in (1, 2, 3):
        v = np.arange(1 << (8 * L), dtype=np.uint32)
        groups.append(np.stack([(v >> (8 * k)) & 0xFF for k in range(L)], axis=1).astype(np.uint8))
    arena, in_off, in_len = _layout(groups, 1)
    assert in_off.size == 16_843_008
    assert set((in_off[in_len == 3] % 16).tolist()) == set(range(16))
    n_ok = _run_batch(ctx, arena, in_off, in_len, 0, "all strings of <= 3 bytes")
    assert n_ok == 128 + 18304 + 2650112  # V(1) + V(2) + V(3)
    words = np.arange(65536, dtype=np.uint16)[:, None]
    arena, in_off, in_len = _layout([words], 2)
    n_ok = _run_batch(ctx, arena, in_off, in_len, 1, "all single UTF-16 words")
    assert n_ok == 65536 - 2048


def test_class_alphabets_to_length_5(ctx):
    groups = [_all_strings(ALPHA8, L).astype(np.uint8) for L in range(1, 6)]
    arena, in_off, in_len = _layout(groups, 1)
    assert in_off.size == sum(26 ** L for L in range(1, 6))
    _run_batch(ctx, arena, in_off, in_len, 0, "UTF-8 class alphabet to length 5")
    groups = [_all_strings(ALPHA16, L).astype(np.uint16) for L in range(1, 6)]
    arena, in_off, in_len = _layout(groups, 2)
    _run_batch(ctx, arena, in_off, in_len, 1, "UTF-16 class alphabet to length 5")


def test_class_alphabet_single_buffer_calls_at_every_phase(ctx):
    """Each string of up to 3 class-edge bytes through its own single-buffer calls
    (transcode, validate, length query), string k placed at byte phase k mod 16 of the
    chunk grid; results collected on the device and compared with the oracle."""
    import torch

    strs = [s for L in (1, 2, 3) for s in _all_strings(ALPHA8, L).astype(np.uint8)]
    n = len(strs)
    slot = 32  # bytes per string in the input buffer: 16 of phase + up to 3 bytes + spare
    buf = np.zeros(n * slot + 64, dtype=np.uint8)
    for k, s in enumerate(strs):
        buf[k * slot + k % 16:k * slot + k % 16 + s.size] = s
    d_buf = torch.from_numpy(buf).cuda()
    d_out = torch.full((n * 4,), 0x5A5A, dtype=torch.int16, device="cuda")  # 3 words + guard each
    res = utfx.result_tensor(3 * n)
    note("single-buffer class alphabet: %d strings x 3 calls" % n)
    for k, s in enumerate(strs):
        a = k * slot + k % 16
        src = d_buf[a:a + s.size]
        assert ctx.utf8_to_utf16le_async(src, d_out[4 * k:4 * k + s.size], res[72 * k:72 * k + 24]) == utfx.OK
        assert ctx.validate_utf8_async(src, res[72 * k + 24:72 * k + 48]) == utfx.OK
        assert ctx.utf16_length_from_utf8_async(src, res[72 * k + 48:72 * k + 72]) == utfx.OK
    torch.cuda.synchronize()
    got = utfx.results_from_tensor(res)
    out = d_out.cpu().numpy().view(np.uint16).reshape(n, 4)
    for k, s in enumerate(strs):
        want, ref = O.utf8_to_utf16le(s)
        assert tuple(got[3 * k]) == tuple(want), (s.tobytes().hex(), k % 16, got[3 * k], want)
        assert np.array_equal(out[k, :want.written], ref[:want.written]), (s.tobytes().hex(), k % 16)
        assert np.all(out[k, s.size:] == 0x5A5A)
        assert tuple(got[3 * k + 1]) == tuple(O.validate_utf8(s))
        assert tuple(got[3 * k + 2]) == tuple(O.utf16_length_from_utf8(s))


def _oracle_slice(values, utf16, pool, workers, st, ct, wr):
    """Per-string status, count and written (into st, ct, wr) of the oracle on the 2^24
    four-byte strings whose little-endian bytes are `values` (uint32), in parallel
    chunks.  Returns the number of valid strings."""
    buf = values.view(np.uint8)
    n = values.size
    step = (n + workers - 1) // workers

    def part(lo):
        hi = min(n, lo + step)
        b = buf[4 * lo:4 * hi]
        out = (st[lo:hi], ct[lo:hi], wr[lo:hi])
        if utf16:
            return O.transcode_fixed(b.view(np.uint16), 2, utf16_in=True, out=out)[0]
        return O.transcode_fixed(b, 4, out=out)[0]

    return sum(pool.map(part, range(0, n, step)))


def _exhaustive_4byte(ctx, direction):
    import torch

    S = 1 << 24
    n_slices = 1 << 8
    workers = _workers()
    i = torch.arange(S, dtype=torch.int64, device="cuda")
    out_unit = 4 if direction == 0 else 6  # output room per string, in output units
    out_bytes_per = 8 if direction == 0 else 6
    items = torch.empty((S, 5), dtype=torch.int64, device="cuda")
    items[:, 1] = 4 if direction == 0 else 2
    items[:, 2] = i * out_bytes_per
    items[:, 3] = out_unit
    items[:, 4] = direction
    d_items = items.view(torch.uint8).view(-1)
    arena = torch.zeros(S * 4 + 64, dtype=torch.uint8, device="cuda")
    d_out = torch.empty(S * out_bytes_per + 64, dtype=torch.uint8, device="cuda")
    res = utfx.result_tensor(S)
    res64 = res.view(torch.int64).view(S, 3)
    valid = 0
    st = np.empty(S, dtype=np.int32)
    ct = np.empty(S, dtype=np.uint64)
    wr = np.empty(S, dtype=np.uint64)
    with cf.ThreadPoolExecutor(workers) as pool:
        for s in range(n_slices):
            phase = (s % 12) if direction == 0 else 2 * (s % 6)  # byte phase of the first string
            v = i + (s << 24)
            arena[phase:phase + 4 * S] = torch.stack([(v >> (8 * k)) & 0xFF for k in range(4)], dim=1).to(
                torch.uint8).view(-1)
            items[:, 0] = i * 4 + phase
            if s % 32 == 0:
                note("exhaustive %s: slice %d of %d" % ("utf8 4-byte" if direction == 0 else "utf16 pairs", s,
                                                        n_slices))
            assert ctx.batch_run(arena, d_out, d_items, S, S * (4 if direction == 0 else 2), res) == utfx.OK
            gpu = torch.stack([res64[:, 0] & 0xFFFFFFFF, res64[:, 1], res64[:, 2]], dim=0).to(torch.uint8)
            vals = np.arange(S, dtype=np.uint32) + np.uint32(s << 24)
            nv = _oracle_slice(vals, direction == 1, pool, workers, st, ct, wr)
            g = gpu.cpu().numpy()  # rows: status, count, written
            for row, want in ((0, st), (1, ct), (2, wr)):
                w8 = want.astype(np.uint8)
                if not np.array_equal(g[row], w8):
                    bad = np.nonzero(g[row] != w8)[0][:5]
                    assert False, (s, row, bad, vals[bad], g[:, bad], st[bad], ct[bad], wr[bad])
            assert int(np.count_nonzero(g[0] == 0)) == nv
            valid += nv
    return valid


def test_all_four_byte_utf8_strings(ctx):
    assert _exhaustive_4byte(ctx, 0) == 383_270_912


def test_all_utf16_word_pairs(ctx):
    assert _exhaustive_4byte(ctx, 1) == 63488 ** 2 + 1024 ** 2 == 4_031_774_720
