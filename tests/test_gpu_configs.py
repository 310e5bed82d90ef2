"""Parity at the configured workloads' own sizes.

* The batched workload exactly as the benchmark times it: 200,000 strings, log-normal
  lengths (median 256 B, sigma 2, 8 B .. 4 MiB), mixed profiles and directions, 0.5 %
  with one injected error.  Every item's status, count and written, its output prefix,
  and every byte outside the output slots, against the oracle's batched reference
  (each item = the single-string call on its bytes): once eagerly and on three
  replays of a captured graph, with eager work between the replays.
* Long strings of 4-8 MiB mixed with short ones in one batch: their look-back spans
  more than one 128-segment window of the per-string look-back.
* A graph whose context's workspace was reallocated afterwards is refused, not replayed.
"""
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
    c = utfx.Context()
    yield c
    c.close()


def _compare(got_res, got_out, ora_res, ora_out, items, label):
    compare_batch(got_res, got_out, ora_res, ora_out, items, label, guard=GUARD)


def test_batched_workload_at_full_size_eager_and_graph(ctx):
    import torch

    n = 200_000
    b = synth.make_batch(n, seed_key=(0, 4), median=256, sigma=2.0, hi=4 << 20, err_frac=0.005)
    caps, out_off, out_bytes = synth.batch_output_layout(b)
    items = O.items_array(b.in_off, b.in_len, out_off, caps, b.direction)
    total = int(np.sum(b.in_len))
    note("full batch: %d strings, %d input units, %d output bytes" % (n, total, out_bytes))
    ora_res, ora_out, n_ok = O.batch(b.arena, items, out_bytes)
    n_err = n - n_ok
    # 0.5 % of the strings carry an error: binomial(200000, 0.005) is 1000 +- 31.5
    assert abs(n_err - 1000) < 4 * 31.5, n_err

    d_in = torch.from_numpy(b.arena).cuda()
    d_out = torch.full((out_bytes,), GUARD, dtype=torch.uint8, device="cuda")
    d_items = torch.from_numpy(items.view(np.uint8).copy()).cuda()
    res = utfx.result_tensor(n)
    assert ctx.batch_run(d_in, d_out, d_items, n, total, res) == utfx.OK, ctx.last_error()
    torch.cuda.synchronize()
    _compare(res.cpu().numpy(), d_out.cpu().numpy(), ora_res, ora_out, items, "eager")

    # the same call captured into a graph, replayed three times into cleared buffers,
    # with eager single-buffer work and synchronisations between the replays
    ctx.capture_begin()
    try:
        assert ctx.batch_run(d_in, d_out, d_items, n, total, res) == utfx.OK
    finally:
        g = ctx.capture_end()
    probe = torch.from_numpy(synth.utf8_buffer("cjk", 1 << 20, synth.rng_for(50, 1))).cuda()
    probe_out = torch.empty(1 << 20, dtype=torch.int16, device="cuda")
    for rep in range(3):
        d_out.fill_(GUARD)
        res.zero_()
        torch.cuda.synchronize()
        note("full batch graph replay %d" % rep)
        g.launch()
        torch.cuda.synchronize()
        _compare(res.cpu().numpy(), d_out.cpu().numpy(), ora_res, ora_out, items, "replay %d" % rep)
        r = ctx.utf8_to_utf16le(probe, probe_out)
        assert r.status == utfx.OK
    g.close()


def test_batch_with_multi_window_strings(ctx):
    """Strings of 4-8 MiB (129-257 segments of 32 KiB: the per-string look-back walks
    more than one 128-segment window) among short ones, with errors late in some."""
    import torch

    rng = synth.rng_for(51, 1)
    pieces = []
    for k, (L, prof) in enumerate((((4 << 20) + 7, "cjk"), ((6 << 20) + 1, "emoji"), ((8 << 20) - 3, "mixed4"))):
        d8 = synth.utf8_buffer(prof, L, rng)
        if k == 1:
            d8[L - 100_000] = 0xFF  # error in the last segments
        pieces.append((d8, 0))
        w = synth.utf16_buffer(prof, L // 2, rng)
        if k == 2:
            w[(L // 2) - 50_000] = 0xDC00
        pieces.append((w.astype("<u2").view(np.uint8), 1))
        for _ in range(50):
            s = int(rng.integers(1, 3000))
            pieces.append((synth.utf8_buffer("latin", s, rng), 0))
            pieces.append((synth.utf16_buffer("cjk", s, rng).astype("<u2").view(np.uint8), 1))
    out, in_off, in_len, dirs = [], [], [], []
    off = 0
    for raw, d in pieces:
        pad = int(rng.integers(0, 16))
        if d == 1 and (off + pad) % 2:
            pad += 1
        out.append(np.zeros(pad, np.uint8))
        off += pad
        in_off.append(off)
        in_len.append(raw.size if d == 0 else raw.size // 2)
        dirs.append(d)
        out.append(raw)
        off += raw.size
    out.append(np.zeros(64, np.uint8))
    arena = np.concatenate(out)
    bb = synth.Batch(arena, np.array(in_off, np.uint64), np.array(in_len, np.uint64), np.array(dirs, np.uint32),
                     np.zeros(len(dirs), np.uint8), np.full(len(dirs), -1, np.int64))
    caps, out_off, out_bytes = synth.batch_output_layout(bb)
    items = O.items_array(bb.in_off, bb.in_len, out_off, caps, bb.direction)
    ora_res, ora_out, _ = O.batch(arena, items, out_bytes)
    d_in = torch.from_numpy(arena).cuda()
    d_out = torch.full((out_bytes,), GUARD, dtype=torch.uint8, device="cuda")
    d_items = torch.from_numpy(items.view(np.uint8).copy()).cuda()
    res = utfx.result_tensor(len(dirs))
    note("multi-window batch: %d strings, longest %d units" % (len(dirs), int(bb.in_len.max())))
    assert ctx.batch_run(d_in, d_out, d_items, len(dirs), int(np.sum(bb.in_len)), res) == utfx.OK
    torch.cuda.synchronize()
    _compare(res.cpu().numpy(), d_out.cpu().numpy(), ora_res, ora_out, items, "multi-window")


def test_graph_refused_after_workspace_growth():
    """A graph keeps the workspace addresses of its context: once an eager call has
    reallocated that workspace, replaying the graph is refused on the host."""
    import torch

    with utfx.Context() as c:
        b = synth.make_batch(64, seed_key=(52, 1), median=100, sigma=0.5, hi=1000, err_frac=0.0)
        caps, out_off, out_bytes = synth.batch_output_layout(b)
        items = utfx.pack_items(b.in_off, b.in_len, out_off, caps, b.direction)
        d_in = torch.from_numpy(b.arena).cuda()
        d_out = torch.zeros(out_bytes, dtype=torch.uint8, device="cuda")
        res = utfx.result_tensor(64)
        total = int(np.sum(b.in_len))
        assert c.batch_run(d_in, d_out, items, 64, total, res) == utfx.OK
        torch.cuda.synchronize()
        c.capture_begin()
        try:
            assert c.batch_run(d_in, d_out, items, 64, total, res) == utfx.OK
        finally:
            g = c.capture_end()
        g.launch()  # fine before the workspace grows
        torch.cuda.synchronize()
        big = synth.make_batch(5000, seed_key=(52, 2), median=100, sigma=0.5, hi=1000, err_frac=0.0)
        caps2, out_off2, out_bytes2 = synth.batch_output_layout(big)
        items2 = utfx.pack_items(big.in_off, big.in_len, out_off2, caps2, big.direction)
        d_in2 = torch.from_numpy(big.arena).cuda()
        d_out2 = torch.zeros(out_bytes2, dtype=torch.uint8, device="cuda")
        res2 = utfx.result_tensor(5000)
        assert c.batch_run(d_in2, d_out2, items2, 5000, int(np.sum(big.in_len)), res2) == utfx.OK  # grows
        torch.cuda.synchronize()
        with pytest.raises(utfx.UtfxError):
            g.launch()
        assert "capture it again" in c.last_error()
        g.close()
