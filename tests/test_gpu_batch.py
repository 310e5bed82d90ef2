"""GPU parity of the batched call: every item of a batch gets exactly the result and
output prefix the scalar oracle gives on its bytes (and the single-buffer call), with
nothing stored outside an item's output slot.  Covers both paths (one wave per
string up to 16,384 units, segmented look-back above), their boundary, errors,
capacity limits, bad descriptors and back-to-back calls."""
import numpy as np
import pytest

import oracle as O
import paper_2212_05098_amd as utfx
from paper_2212_05098_amd import synth
from gpu_helpers import note

pytestmark = pytest.mark.gpu

SMALL_MAX = 16384
GUARD = 0xA5


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available()
    c = utfx.Context()
    yield c
    c.close()


def layout_outputs(in_len, dirs, caps, rng):
    """Output offsets with a random gap (>= 8 bytes) before every slot; UTF-16 slots
    start at even addresses."""
    out_off = np.zeros(len(in_len), dtype=np.uint64)
    off = 0
    for i in range(len(in_len)):
        off += 8 + int(rng.integers(0, 9))
        if dirs[i] == 0 and off % 2:
            off += 1
        out_off[i] = off
        off += int(caps[i]) * (2 if dirs[i] == 0 else 1)
    return out_off, off + 64


def run_and_check(ctx, arena, in_off, in_len, dirs, caps, rng, total=None, expect=None):
    """Run one batch and check every item against the oracle.  expect maps item index
    to a forced status (bad descriptors, plan overflow)."""
    import torch

    n = len(in_off)
    out_off, out_size = layout_outputs(in_len, dirs, caps, rng)
    d_in = torch.from_numpy(np.ascontiguousarray(arena, dtype=np.uint8)).cuda()
    d_out = torch.full((out_size,), GUARD, dtype=torch.uint8, device="cuda")
    items = utfx.pack_items(in_off, in_len, out_off, caps, dirs)
    res = utfx.result_tensor(n)
    units = int(np.sum(in_len)) if total is None else total
    note("batch n=%d total_units=%d max_len=%d" % (n, units, int(np.max(in_len)) if n else 0))
    st = ctx.batch_run(d_in, d_out, items, n, units, res)
    assert st == utfx.OK, ctx.last_error()
    torch.cuda.synchronize()
    got = utfx.results_from_tensor(res)
    out = d_out.cpu().numpy()
    used = np.zeros(out_size, dtype=bool)
    expect = expect or {}
    for i in range(n):
        a, L, cap, d = int(in_off[i]), int(in_len[i]), int(caps[i]), int(dirs[i])
        o = int(out_off[i])
        if i in expect:
            assert got[i].status == expect[i], (i, got[i])
            continue
        if d == 0:
            data = arena[a:a + L]
            want, ref = O.utf8_to_utf16le(data, cap=cap)
            w = min(want.written, cap)
            gw = out[o:o + 2 * w].view(np.uint16)
            used[o:o + 2 * cap] = True
        else:
            data = arena[a:a + 2 * L].view(np.uint16)
            want, ref = O.utf16le_to_utf8(data, cap=cap)
            w = min(want.written, cap)
            gw = out[o:o + w]
            used[o:o + cap] = True
        assert tuple(got[i]) == tuple(want), (i, d, L, got[i], want)
        assert np.array_equal(gw, ref[:w]), (i, d, L)
    assert np.all(out[~used] == GUARD), "bytes outside the output slots changed"
    return got


@pytest.mark.parametrize("n", [3000, 6000])
def test_batch_mixed_profiles_and_errors(ctx, n):
    """n strings, log-normal lengths (median 256 B, sigma 2), mixed profiles and
    directions, 5 % with an injected error, random output caps on 5 %.  With 6,000
    strings (calls of 4,096 or more) the tiny ones go through the row kernel."""
    b = synth.make_batch(n, seed_key=(7, 1, n), median=256, sigma=2.0, hi=256 << 10, err_frac=0.05)
    rng = synth.rng_for(7, 2)
    need = np.where(b.direction == 0, b.in_len, 3 * b.in_len).astype(np.uint64)
    caps = need.copy()
    short = rng.random(len(caps)) < 0.05
    caps[short] = (caps[short] * rng.random(int(short.sum()))).astype(np.uint64)
    assert np.sum(b.in_len > SMALL_MAX) >= 5  # both paths are exercised
    run_and_check(ctx, b.arena, b.in_off, b.in_len, b.direction, caps, rng)


def _arena_of(pieces):
    """Concatenate (bytes, dir) pieces with random misalignment; UTF-16 pieces even."""
    rng = synth.rng_for(9, 9)
    out, in_off, in_len, dirs = [], [], [], []
    off = 0
    for raw, d in pieces:
        pad = int(rng.integers(0, 16))
        if d == 1 and (off + pad) % 2:
            pad += 1
        out.append(np.zeros(pad, dtype=np.uint8))
        off += pad
        in_off.append(off)
        in_len.append(raw.size if d == 0 else raw.size // 2)
        dirs.append(d)
        out.append(raw)
        off += raw.size
    out.append(np.zeros(64, dtype=np.uint8))
    return (np.concatenate(out), np.array(in_off, dtype=np.uint64), np.array(in_len, dtype=np.uint64),
            np.array(dirs, dtype=np.uint32))


def test_batch_path_boundary_and_large_errors(ctx):
    """Lengths around the one-wave limit and across several segments of the long-string
    path, with errors at chunk, segment and string ends."""
    rng = synth.rng_for(11, 3)
    pieces = []
    for L in (0, 1, 15, 16, 1023, 1024, 1025, SMALL_MAX - 1, SMALL_MAX, SMALL_MAX + 1, 32768 + 5, 100000,
              300001):
        for prof in ("cjk", "emoji"):
            d8 = synth.utf8_buffer(prof, L, rng)
            pieces.append((d8, 0))
            w = synth.utf16_buffer(prof, L // 2, rng)
            pieces.append((w.astype("<u2").view(np.uint8), 1))
    # errors near the ends of long strings and at a segment edge (32 KiB segments)
    for L, at in ((SMALL_MAX + 1, SMALL_MAX - 2), (70000, 32768 - 1), (70000, 65536 + 1), (200000, 199998)):
        d8 = np.frombuffer(b"a" * L, dtype=np.uint8).copy()
        d8[at] = 0xE2
        pieces.append((d8, 0))
        w = np.full(L // 2, 0x41, dtype=np.uint16)
        w[min(at // 2, w.size - 1)] = 0xD83D
        pieces.append((w.astype("<u2").view(np.uint8), 1))
    arena, in_off, in_len, dirs = _arena_of(pieces)
    caps = np.where(dirs == 0, in_len, 3 * in_len).astype(np.uint64)
    got = run_and_check(ctx, arena, in_off, in_len, dirs, caps, rng)
    # the same items through the single-buffer calls
    import torch

    for i in range(0, len(in_off), 7):
        a, L = int(in_off[i]), int(in_len[i])
        if dirs[i] == 0:
            src = torch.from_numpy(arena[a:a + L].copy()).cuda()
            dst = torch.empty(max(L, 1), dtype=torch.int16, device="cuda")
            r = ctx.utf8_to_utf16le(src, dst[:L])
        else:
            src = torch.from_numpy(arena[a:a + 2 * L].view(np.int16).copy()).cuda()
            dst = torch.empty(max(3 * L, 1), dtype=torch.uint8, device="cuda")
            r = ctx.utf16le_to_utf8(src, dst[:3 * L])
        assert tuple(r) == tuple(got[i]), (i, r, got[i])


def test_batch_bad_descriptors_and_plan_bound(ctx):
    rng = synth.rng_for(12, 1)
    pieces = [(synth.utf8_buffer("latin", 500, rng), 0), (synth.utf8_buffer("cjk", 40000, rng), 0),
              (synth.utf16_buffer("emoji", 300, rng).astype("<u2").view(np.uint8), 1),
              (synth.utf16_buffer("cjk", 30000, rng).astype("<u2").view(np.uint8), 1)]
    arena, in_off, in_len, dirs = _arena_of(pieces)
    caps = np.where(dirs == 0, in_len, 3 * in_len).astype(np.uint64)
    # bad: direction 2; UTF-16 input at an odd address; length above the limit
    bad_dir = dirs.copy()
    bad_dir[0] = 2
    run_and_check(ctx, arena, in_off, in_len, bad_dir, caps, rng, expect={0: utfx.E_INVALID_ARG})
    odd = in_off.copy()
    odd[2] += 1
    run_and_check(ctx, arena, odd, in_len, dirs, caps, rng, expect={2: utfx.E_INVALID_ARG})
    # a plan bound far below the real total: the long strings report INVALID_ARG,
    # the short ones are unaffected
    run_and_check(ctx, arena, in_off, in_len, dirs, caps, rng, total=10,
                  expect={1: utfx.E_INVALID_ARG, 3: utfx.E_INVALID_ARG})


def test_batch_back_to_back(ctx):
    """Two calls in a row on the same context with different contents and sizes."""
    for k, n in ((1, 800), (2, 300)):
        b = synth.make_batch(n, seed_key=(13, k), median=2048, sigma=1.5, hi=128 << 10, err_frac=0.1)
        rng = synth.rng_for(13, k, 5)
        caps = np.where(b.direction == 0, b.in_len, 3 * b.in_len).astype(np.uint64)
        run_and_check(ctx, b.arena, b.in_off, b.in_len, b.direction, caps, rng)


@pytest.mark.parametrize("tuning", [(1024, 2, 1), (4096, 4, 1), (65536, 2, 2), (262144, 4, 2)])
def test_batch_tunings_same_results(tuning):
    """Every batch tuning (longest wave-walked string, segment tiles, persistent
    segment workgroups per CU) gives the oracle's results on the same batch: strings up
    to 1 MiB, 5 % with errors, caps cut on 5 %."""
    b = synth.make_batch(4000, seed_key=(7, 5), median=512, sigma=2.5, hi=1 << 20, err_frac=0.05)
    rng = synth.rng_for(7, 6)
    caps = np.where(b.direction == 0, b.in_len, 3 * b.in_len).astype(np.uint64)
    short = rng.random(len(caps)) < 0.05
    caps[short] = (caps[short] * rng.random(int(short.sum()))).astype(np.uint64)
    with utfx.Context() as c:
        c.set_batch_tuning(*tuning)
        assert c.get_batch_tuning() == tuning
        note("batch tuning %s" % (tuning,))
        run_and_check(c, b.arena, b.in_off, b.in_len, b.direction, caps, rng)
        with pytest.raises(utfx.UtfxError):
            c.set_batch_tuning(512, 4, 2)
        # the wave walkers keep positions in 32 bits on the strength of this bound
        with pytest.raises(utfx.UtfxError):
            c.set_batch_tuning((1 << 18) + 1, 4, 2)
