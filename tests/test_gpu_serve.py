"""The continuous-batching server: every request served through it (host payload in,
host output out) matches the oracle exactly, whether it was batched with others or
alone; small arenas force admission to wait; oversized requests are rejected."""
import numpy as np
import pytest

import oracle as O
import paper_2212_05098_amd as utfx
from paper_2212_05098_amd import serve, synth
from gpu_helpers import note

pytestmark = pytest.mark.gpu


def _check(data, d, out_bytes, res):
    if d == 0:
        want, ref = O.utf8_to_utf16le(data)
        got = out_bytes[:2 * want.written].view(np.uint16)
    else:
        want, ref = O.utf16le_to_utf8(data)
        got = out_bytes[:want.written]
    assert tuple(res) == tuple(want), (d, res, want)
    assert np.array_equal(got, ref[:want.written])


def test_server_progress_small_arenas():
    """500 requests through arenas of 64 KiB: most steps are full, requests wait for
    admission; one request larger than an arena completes with INVALID_ARG."""
    rng = synth.rng_for(31, 1)
    srv = utfx.Server(arena_in_bytes=64 << 10, arena_out_bytes=192 << 10, max_items=64, inflight=2)
    reqs = []
    for i in range(500):
        d = int(rng.integers(0, 2))
        prof = synth.SCRIPT_PROFILES[int(rng.integers(0, 4))]
        L = int(synth.lognormal_lengths(rng, 1, 300, 1.5, 1, 30000)[0])
        if d == 0:
            data = synth.utf8_buffer(prof, L, rng)
            if rng.random() < 0.1 and L > 4:
                data[int(rng.integers(0, L))] = 0xC0
            cap = data.size
            out = np.zeros(2 * cap + 2, dtype=np.uint8)
        else:
            data = synth.utf16_buffer(prof, max(L // 2, 1), rng)
            if rng.random() < 0.1:
                data[int(rng.integers(0, data.size))] = 0xD800
            cap = 3 * data.size
            out = np.zeros(cap + 1, dtype=np.uint8)
        reqs.append((data, d, cap, out))
    big = np.full(100 << 10, 0x41, dtype=np.uint8)
    big_out = np.zeros(2 * big.size, dtype=np.uint8)
    reqs.append((big, 0, big.size, big_out))
    for i, (data, d, cap, out) in enumerate(reqs):
        n_units = data.size
        assert srv.submit(i, data.ctypes.data, n_units, d, out.ctypes.data, cap) == utfx.OK
    got = {}
    note("server progress: %d requests" % len(reqs))
    for _ in range(2_000_000):
        for tag, r in srv.progress():
            got[tag] = r
        if len(got) == len(reqs):
            break
    assert len(got) == len(reqs)
    assert got[len(reqs) - 1].status == utfx.E_INVALID_ARG
    for i, (data, d, cap, out) in enumerate(reqs[:-1]):
        _check(data, d, out, got[i])
    srv.close()


def test_server_replay_trace_fully_checked():
    """A seeded Poisson trace (20k requests/s for 0.25 s) replayed in real time with
    every request checked against the oracle."""
    import torch

    pool = serve.PayloadPool(mib_per_pool=4, seed=1)
    check = torch.zeros(256 << 20, dtype=torch.uint8, pin_memory=True)
    scratch = torch.zeros(64 << 20, dtype=torch.uint8, pin_memory=True)
    w = serve.make_workload(pool, 20000, 0.25, seed=3, scratch_ptr=scratch.data_ptr(), check_every=1,
                            check_ptr=check.data_ptr(), check_bytes=check.numel())
    assert w.checked.size > 0.9 * w.arrival_ns.size
    srv = utfx.Server(arena_in_bytes=64 << 20, arena_out_bytes=192 << 20, max_items=65536, inflight=2)
    note("server replay: %d requests" % w.arrival_ns.size)
    lat, res, wall = srv.replay(w.arrival_ns, w.data_ptrs, w.len_units, w.dirs, w.out_ptrs, w.out_caps)
    srv.close()
    assert np.all(lat > 0)
    outs = check.numpy()
    import ctypes

    for j, i in enumerate(w.checked):
        d, n = int(w.dirs[i]), int(w.len_units[i])
        raw = np.ctypeslib.as_array((ctypes.c_uint8 * (n * (2 if d else 1))).from_address(int(w.data_ptrs[i])))
        data = raw.view(np.uint16) if d else raw
        r = utfx.Result(int(res[i]["status"]), int(res[i]["count"]), int(res[i]["written"]))
        _check(data, d, outs[int(w.check_off[j]):], r)


def test_server_bulk_and_direct_requests():
    """Small requests interleaved with bulk ones (1 MiB of input or more), pageable and
    pinned host buffers (staged and direct copies), one bulk request with an error and
    one larger than the arenas: every request matches the oracle, the oversized one is
    rejected."""
    import torch

    rng = synth.rng_for(31, 2)
    srv = utfx.Server(arena_in_bytes=8 << 20, arena_out_bytes=24 << 20, max_items=256, inflight=3)
    reqs, keep = [], []
    for i in range(60):
        d = i % 2
        prof = synth.SCRIPT_PROFILES[i % 4]
        bulk = i % 10 in (3, 6)
        pinned = i % 4 < 2
        n = int(rng.integers(1 << 20, 3 << 20)) if bulk else int(rng.integers(1, 5000))
        if d == 0:
            data = synth.utf8_buffer(prof, n, rng)
            if i == 16:
                data[n // 2] = 0xFF
            cap, ob = data.size, 2 * data.size + 2
        else:
            data = synth.utf16_buffer(prof, max(n // 2, 1), rng)
            if i == 23:
                data[data.size // 3 - 1:data.size // 3 + 1] = (0x41, 0xDC00)
            cap, ob = 3 * data.size, 3 * data.size + 1
        if pinned:
            t_in = torch.from_numpy(data.view(np.uint8).copy()).pin_memory()
            t_out = torch.zeros(ob, dtype=torch.uint8).pin_memory()
            keep += [t_in, t_out]
            in_ptr, out_arr, out_ptr = t_in.data_ptr(), t_out.numpy(), t_out.data_ptr()
        else:
            out_arr = np.zeros(ob, dtype=np.uint8)
            in_ptr, out_ptr = data.ctypes.data, out_arr.ctypes.data
        reqs.append((data, d, cap, out_arr))
        assert srv.submit(i, in_ptr, data.size, d, out_ptr, cap) == utfx.OK
    big = np.full(9 << 20, 0x41, dtype=np.uint8)
    big_out = np.zeros(2 * big.size, dtype=np.uint8)
    assert srv.submit(len(reqs), big.ctypes.data, big.size, 0, big_out.ctypes.data, big.size) == utfx.OK
    note("server bulk/direct: %d requests" % (len(reqs) + 1))
    got = {}
    for _ in range(5_000_000):
        for tag, r in srv.progress():
            got[tag] = r
        if len(got) == len(reqs) + 1:
            break
    assert len(got) == len(reqs) + 1
    assert got[len(reqs)].status == utfx.E_INVALID_ARG
    assert got[16].status != utfx.OK and got[23].status == utfx.E_SURROGATE
    for i, (data, d, cap, out) in enumerate(reqs):
        _check(data, d, out, got[i])
    srv.close()


def test_server_device_cap():
    with pytest.raises(utfx.UtfxError):
        utfx.Server(arena_in_bytes=1 << 30, arena_out_bytes=2 << 30, inflight=2, device_cap_bytes=4 << 30)


def test_device_resident_requests_mixed_with_host_requests():
    """Device-resident requests (payload and output in device memory, flag
    SERVER_DEVICE_BUFFERS) served in the same steps as host requests: every result and
    output matches the oracle, and the device outputs leave the bytes after their valid
    prefix untouched."""
    import torch

    rng = synth.rng_for(31, 7)
    srv = utfx.Server(arena_in_bytes=1 << 20, arena_out_bytes=3 << 20, max_items=256, inflight=3)
    reqs = []
    for i in range(600):
        d = int(rng.integers(0, 2))
        prof = synth.SCRIPT_PROFILES[int(rng.integers(0, 4))]
        L = int(synth.lognormal_lengths(rng, 1, 500, 2.0, 1, 200000)[0])
        if d == 0:
            data = synth.utf8_buffer(prof, L, rng)
            if rng.random() < 0.1 and L > 4:
                data[int(rng.integers(0, L))] = 0xFF
            cap, out_len = data.size, 2 * data.size
        else:
            data = synth.utf16_buffer(prof, max(L // 2, 1), rng)
            if rng.random() < 0.1:
                data[int(rng.integers(0, data.size))] = 0xDC00
            cap, out_len = 3 * data.size, 3 * data.size
        dev = bool(rng.random() < 0.6)
        if dev:
            raw = data.view(np.uint8)
            shift = int(rng.integers(0, 16)) & (~1 if d == 1 else ~0)  # any start; UTF-16 stays 2-byte aligned
            src_t = torch.zeros(raw.size + 32, dtype=torch.uint8, device="cuda")
            src_t[shift:shift + raw.size] = torch.from_numpy(raw.copy()).cuda()
            out_t = torch.full((out_len + 32,), 0xA5, dtype=torch.uint8, device="cuda")
            reqs.append((data, d, cap, out_t, src_t, shift, True))
        else:
            reqs.append((data, d, cap, np.zeros(out_len + 2, dtype=np.uint8), None, 0, False))
    torch.cuda.synchronize()
    for i, (data, d, cap, out, src_t, shift, dev) in enumerate(reqs):
        if dev:
            st = srv.submit(i, src_t.data_ptr() + shift, data.size, d | utfx.SERVER_DEVICE_BUFFERS, out.data_ptr(),
                            cap)
        else:
            st = srv.submit(i, data.ctypes.data, data.size, d, out.ctypes.data, cap)
        assert st == utfx.OK
    got = {}
    note("server with device-resident requests: %d requests" % len(reqs))
    for _ in range(2_000_000):
        for tag, r in srv.progress():
            got[tag] = r
        if len(got) == len(reqs):
            break
    assert len(got) == len(reqs)
    for i, (data, d, cap, out, src_t, shift, dev) in enumerate(reqs):
        if dev:
            host = out.cpu().numpy()
            _check(data, d, host, got[i])
            w = got[i].written * (2 if d == 0 else 1)
            assert np.all(host[w:] == 0xA5), i
        else:
            _check(data, d, out, got[i])
    srv.close()
