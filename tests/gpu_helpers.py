"""Helpers shared by the GPU tests: device upload, oracle comparison, progress notes."""
import sys

import numpy as np

import oracle as O


def note(msg):
    """Name the case on the real stderr before a GPU step (survives a crashed run)."""
    sys.__stderr__.write("[gpu-case] %s\n" % msg)
    sys.__stderr__.flush()


def dev_u8(a, pad_front=0, pad_back=0):
    """Upload bytes; returns (tensor_view, backing).  pad_front shifts the start
    address by that many bytes (misalignment tests)."""
    import torch

    a = np.ascontiguousarray(a, dtype=np.uint8)
    back = torch.zeros(pad_front + a.size + pad_back + 16, dtype=torch.uint8, device="cuda")
    if a.size:
        back[pad_front:pad_front + a.size] = torch.from_numpy(a.copy()).cuda()
    return back[pad_front:pad_front + a.size], back


def dev_u16(w, pad_front_words=0, pad_back=0):
    """Upload UTF-16 words as an int16 tensor view (2-byte aligned, shifted by
    pad_front_words words)."""
    import torch

    w = np.ascontiguousarray(w, dtype=np.uint16)
    back = torch.zeros(pad_front_words + w.size + pad_back + 8, dtype=torch.int16, device="cuda")
    if w.size:
        back[pad_front_words:pad_front_words + w.size] = torch.from_numpy(w.view(np.int16).copy()).cuda()
    return back[pad_front_words:pad_front_words + w.size], back


def host_u16(t):
    return t.cpu().numpy().view(np.uint16)


def host_u8(t):
    return t.cpu().numpy().view(np.uint8)


def check_u8_to_u16(ctx, data, cap=None, in_shift=0, out_shift=0, guard=64):
    """Run the GPU transcode and the oracle on the same bytes; compare status, count,
    written, out[:written] and that nothing at or beyond cap changed."""
    import torch

    data = np.ascontiguousarray(data, dtype=np.uint8)
    n = data.size
    cap = n if cap is None else cap
    src, _ = dev_u8(data, pad_front=in_shift)
    fill = 0x5A5A
    out_back = torch.full((out_shift + cap + guard,), fill - 0x10000 if fill > 0x7FFF else fill,
                          dtype=torch.int16, device="cuda")
    dst = out_back[out_shift:out_shift + cap]
    r = ctx.utf8_to_utf16le(src, dst)
    want, ref = O.utf8_to_utf16le(data, cap=cap)
    assert tuple(r) == tuple(want), (r, want)
    got = host_u16(out_back)
    w = min(r.written, cap)
    assert np.array_equal(got[out_shift:out_shift + w], ref[:w])
    assert np.all(got[:out_shift] == fill) and np.all(got[out_shift + cap:] == fill)
    v = ctx.validate_utf8(src)
    vw = O.validate_utf8(data)
    assert tuple(v) == tuple(vw), (v, vw)
    ln = ctx.utf16_length_from_utf8(src)
    assert tuple(ln) == tuple(O.utf16_length_from_utf8(data))
    return r


def check_u16_to_u8(ctx, words, cap=None, in_shift=0, out_shift=0, guard=64):
    import torch

    words = np.ascontiguousarray(words, dtype=np.uint16)
    n = words.size
    cap = 3 * n if cap is None else cap
    src, _ = dev_u16(words, pad_front_words=in_shift)
    out_back = torch.full((out_shift + cap + guard,), 0xA5, dtype=torch.uint8, device="cuda")
    dst = out_back[out_shift:out_shift + cap]
    r = ctx.utf16le_to_utf8(src, dst)
    want, ref = O.utf16le_to_utf8(words, cap=cap)
    assert tuple(r) == tuple(want), (r, want)
    got = host_u8(out_back)
    w = min(r.written, cap)
    assert np.array_equal(got[out_shift:out_shift + w], ref[:w])
    assert np.all(got[:out_shift] == 0xA5) and np.all(got[out_shift + cap:] == 0xA5)
    v = ctx.validate_utf16le(src)
    assert tuple(v) == tuple(O.validate_utf16le(words))
    ln = ctx.utf8_length_from_utf16le(src)
    assert tuple(ln) == tuple(O.utf8_length_from_utf16le(words))
    return r


def check_u8_to_u16be(ctx, data, cap=None, in_shift=0, out_shift=0, guard=64):
    """UTF-8 -> UTF-16BE on the GPU against the oracle; `out` compared as the bytes
    in memory, and nothing written outside [0, cap)."""
    import torch

    data = np.ascontiguousarray(data, dtype=np.uint8)
    cap = data.size if cap is None else cap
    src, _ = dev_u8(data, pad_front=in_shift)
    out_back = torch.full((out_shift + cap + guard,), 0x5A5A, dtype=torch.int16, device="cuda")
    dst = out_back[out_shift:out_shift + cap]
    r = ctx.utf8_to_utf16be(src, dst)
    want, ref = O.utf8_to_utf16be(data, cap=cap)
    assert tuple(r) == tuple(want), (r, want)
    got = host_u16(out_back)
    w = min(r.written, cap)
    assert np.array_equal(got[out_shift:out_shift + w], ref[:w])
    assert np.all(got[:out_shift] == 0x5A5A) and np.all(got[out_shift + cap:] == 0x5A5A)
    return r


def check_u16be_to_u8(ctx, words_be, cap=None, in_shift=0, out_shift=0, guard=64):
    """`words_be` is the UTF-16BE buffer as the uint16 array that holds its bytes."""
    import torch

    words_be = np.ascontiguousarray(words_be, dtype=np.uint16)
    cap = 3 * words_be.size if cap is None else cap
    src, _ = dev_u16(words_be, pad_front_words=in_shift)
    out_back = torch.full((out_shift + cap + guard,), 0xA5, dtype=torch.uint8, device="cuda")
    dst = out_back[out_shift:out_shift + cap]
    r = ctx.utf16be_to_utf8(src, dst)
    want, ref = O.utf16be_to_utf8(words_be, cap=cap)
    assert tuple(r) == tuple(want), (r, want)
    got = host_u8(out_back)
    w = min(r.written, cap)
    assert np.array_equal(got[out_shift:out_shift + w], ref[:w])
    assert np.all(got[:out_shift] == 0xA5) and np.all(got[out_shift + cap:] == 0xA5)
    assert tuple(ctx.validate_utf16be(src)) == tuple(O.validate_utf16be(words_be))
    assert tuple(ctx.utf8_length_from_utf16be(src)) == tuple(O.utf8_length_from_utf16be(words_be))
    return r


def dev_u32(u, pad_front_units=0, pad_back=0):
    """Upload UTF-32 units as an int32 tensor view (4-byte aligned, shifted by
    pad_front_units units)."""
    import torch

    u = np.ascontiguousarray(u, dtype=np.uint32)
    back = torch.zeros(pad_front_units + u.size + pad_back + 4, dtype=torch.int32, device="cuda")
    if u.size:
        back[pad_front_units:pad_front_units + u.size] = torch.from_numpy(u.view(np.int32).copy()).cuda()
    return back[pad_front_units:pad_front_units + u.size], back


def check_u8_to_u32(ctx, data, cap=None, in_shift=0, out_shift=0, guard=32):
    import torch

    data = np.ascontiguousarray(data, dtype=np.uint8)
    cap = data.size if cap is None else cap
    src, _ = dev_u8(data, pad_front=in_shift)
    fill = 0x5A5A5A5A
    out_back = torch.full((out_shift + cap + guard,), fill, dtype=torch.int32, device="cuda")
    dst = out_back[out_shift:out_shift + cap]
    r = ctx.utf8_to_utf32le(src, dst)
    want, ref = O.utf8_to_utf32le(data, cap=cap)
    assert tuple(r) == tuple(want), (r, want)
    got = out_back.cpu().numpy().view(np.uint32)
    w = min(r.written, cap)
    assert np.array_equal(got[out_shift:out_shift + w], ref[:w])
    assert np.all(got[:out_shift] == fill) and np.all(got[out_shift + cap:] == fill)
    return r


def check_u32_to_u8(ctx, units, cap=None, in_shift=0, out_shift=0, guard=64):
    import torch

    units = np.ascontiguousarray(units, dtype=np.uint32)
    cap = 4 * units.size if cap is None else cap
    src, _ = dev_u32(units, pad_front_units=in_shift)
    out_back = torch.full((out_shift + cap + guard,), 0xA5, dtype=torch.uint8, device="cuda")
    dst = out_back[out_shift:out_shift + cap]
    r = ctx.utf32le_to_utf8(src, dst)
    want, ref = O.utf32le_to_utf8(units, cap=cap)
    assert tuple(r) == tuple(want), (r, want)
    got = host_u8(out_back)
    w = min(r.written, cap)
    assert np.array_equal(got[out_shift:out_shift + w], ref[:w])
    assert np.all(got[:out_shift] == 0xA5) and np.all(got[out_shift + cap:] == 0xA5)
    assert tuple(ctx.validate_utf32le(src)) == tuple(O.validate_utf32le(units))
    return r


def check_u16_to_u32(ctx, words, cap=None, in_shift=0, out_shift=0, guard=32, be=False):
    """be: `words` is a UTF-16BE buffer (the uint16 array holding its bytes)."""
    import torch

    words = np.ascontiguousarray(words, dtype=np.uint16)
    cap = words.size if cap is None else cap
    src, _ = dev_u16(words, pad_front_words=in_shift)
    fill = 0x5A5A5A5A
    out_back = torch.full((out_shift + cap + guard,), fill, dtype=torch.int32, device="cuda")
    fn = ctx.utf16be_to_utf32le if be else ctx.utf16le_to_utf32le
    r = fn(src, out_back[out_shift:out_shift + cap])
    want, ref = (O.utf16be_to_utf32le if be else O.utf16le_to_utf32le)(words, cap=cap)
    assert tuple(r) == tuple(want), (r, want)
    got = out_back.cpu().numpy().view(np.uint32)
    w = min(r.written, cap)
    assert np.array_equal(got[out_shift:out_shift + w], ref[:w])
    assert np.all(got[:out_shift] == fill) and np.all(got[out_shift + cap:] == fill)
    return r


def check_u32_to_u16(ctx, units, cap=None, in_shift=0, out_shift=0, guard=32, be=False):
    """be: the output is UTF-16BE (compared as the bytes in memory)."""
    import torch

    units = np.ascontiguousarray(units, dtype=np.uint32)
    cap = 2 * units.size if cap is None else cap
    src, _ = dev_u32(units, pad_front_units=in_shift)
    out_back = torch.full((out_shift + cap + guard,), 0x5A5A, dtype=torch.int16, device="cuda")
    fn = ctx.utf32le_to_utf16be if be else ctx.utf32le_to_utf16le
    r = fn(src, out_back[out_shift:out_shift + cap])
    want, ref = (O.utf32le_to_utf16be if be else O.utf32le_to_utf16le)(units, cap=cap)
    assert tuple(r) == tuple(want), (r, want)
    got = host_u16(out_back)
    w = min(r.written, cap)
    assert np.array_equal(got[out_shift:out_shift + w], ref[:w])
    assert np.all(got[:out_shift] == 0x5A5A) and np.all(got[out_shift + cap:] == 0x5A5A)
    return r


def spans(starts, lengths, size):
    """Boolean mask of the union of [start, start + length) over the items."""
    d = np.zeros(size + 1, dtype=np.int32)
    np.add.at(d, np.asarray(starts).astype(np.int64), 1)
    np.add.at(d, (np.asarray(starts) + np.asarray(lengths)).astype(np.int64), -1)
    return np.cumsum(d[:-1]) > 0


def compare_batch(got_res, got_out, ora_res, ora_out, items, label, guard=None):
    """A batched call against the oracle's batched reference, vectorised: every item's
    status, count and written; every byte of every output prefix; and, with `guard`,
    that every byte outside the output slots still holds the guard value."""
    g = np.ascontiguousarray(got_res).view(np.uint8).view(O.RESULT_DTYPE)
    for f in ("status", "count", "written"):
        bad = np.nonzero(g[f] != ora_res[f])[0]
        assert bad.size == 0, (label, f, bad[:5], g[bad[:5]], ora_res[bad[:5]], items[bad[:5]])
    unit = np.where(items["dir"] == 0, 2, 1).astype(np.uint64)
    w = np.minimum(ora_res["written"], items["out_cap"]) * unit
    w[ora_res["status"] == O.E_OUTPUT_TOO_SMALL] = 0
    m = spans(items["out_off"], w, got_out.size)
    diff = np.nonzero(got_out[m] != ora_out[m])[0]
    assert diff.size == 0, (label, "output bytes differ", diff[:5])
    if guard is not None:
        slots = spans(items["out_off"], items["out_cap"] * unit, got_out.size)
        assert np.all(got_out[~slots] == guard), (label, "stored outside the output slots")
