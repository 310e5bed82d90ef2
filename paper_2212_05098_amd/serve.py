"""Serving workload over the native continuous-batching server (utfx_server_*).

Requests arrive as a seeded Poisson process with log-normal sizes (median 1 KiB,
sigma 2.5, clipped to 8 B .. 16 MiB), mixed script profiles and directions; their
payloads are slices of a pre-generated pinned host pool (cut at character
boundaries, so requests are valid text).  utfx_server_replay submits each request at
its arrival time and drives the server until all complete; latency runs from arrival
to result and output on the host (PCIe included).  A sample of the requests gets its
own output buffer so that the caller can check it; the others share
a scratch output region.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from paper_2212_05098_amd import synth


@dataclass
class Workload:
    arrival_ns: np.ndarray
    data_ptrs: np.ndarray
    len_units: np.ndarray
    dirs: np.ndarray
    out_ptrs: np.ndarray
    out_caps: np.ndarray
    in_bytes: np.ndarray
    checked: np.ndarray          # indices with their own output buffer
    check_off: np.ndarray        # byte offset of each checked request's output buffer


class PayloadPool:
    """Pinned host text per (direction, profile), with the positions where a
    character starts."""

    def __init__(self, mib_per_pool: int = 32, seed: int = 0):
        import torch

        self.buf = {}
        self.starts = {}
        n = mib_per_pool << 20
        for d in (0, 1):
            for p, prof in enumerate(synth.SCRIPT_PROFILES):
                host = synth.config_buffer(prof, d, n, config=5 + seed)
                raw = host.view(np.uint8)
                t = torch.empty(raw.size, dtype=torch.uint8, pin_memory=True)
                t.numpy()[:] = raw
                self.buf[(d, p)] = t
                if d == 0:
                    ok = (raw & 0xC0) != 0x80                     # not a continuation byte
                else:
                    w = raw.view(np.uint16)
                    ok = (w & 0xFC00) != 0xDC00                   # not a low surrogate
                self.starts[(d, p)] = np.flatnonzero(ok).astype(np.int64)

    def slices(self, d: int, p: int, size_bytes: np.ndarray, rng: np.random.Generator):
        """(pointers, lengths in units) of len(size_bytes) slices that start and end
        at character boundaries."""
        t = self.buf[(d, p)]
        st = self.starts[(d, p)]
        unit = 1 if d == 0 else 2
        total = t.numel() // unit
        want = np.minimum(size_bytes // unit, total - 1).astype(np.int64)
        want = np.maximum(want, 1)
        a = (rng.random(want.size) * (total - want)).astype(np.int64)
        a = st[np.minimum(np.searchsorted(st, a), st.size - 1)]          # snap start forward
        e = np.minimum(a + want, total)
        k = np.searchsorted(st, e, side="right") - 1                       # snap end back
        e = np.where(e >= total, total, st[np.maximum(k, 0)])
        e = np.maximum(e, a)
        return t.data_ptr() + a * unit, (e - a)


def make_workload(pool: PayloadPool, rate: float, duration_s: float, seed: int, scratch_ptr: int,
                  check_every: int, check_ptr: int, check_bytes: int) -> Workload:
    tr = synth.poisson_trace(rate, duration_s, seed_key=(0, 5, seed))
    n = tr.arrival_s.size
    rng = synth.rng_for(0, 6, seed, int(rate))
    data_ptrs = np.zeros(n, dtype=np.uint64)
    lens = np.zeros(n, dtype=np.uint64)
    for d in (0, 1):
        for p in range(len(synth.SCRIPT_PROFILES)):
            m = (tr.direction == d) & (tr.profile == p)
            if m.any():
                ptr, ln = pool.slices(d, p, tr.size_bytes[m], rng)
                data_ptrs[m] = ptr
                lens[m] = ln
    dirs = tr.direction.astype(np.uint32)
    out_caps = np.where(dirs == 0, lens, 3 * lens).astype(np.uint64)      # always large enough
    out_bytes = np.where(dirs == 0, 2 * out_caps, out_caps)
    out_ptrs = np.full(n, scratch_ptr, dtype=np.uint64)
    checked = np.arange(0, n, check_every, dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(out_bytes[checked] + 16)[:-1]]).astype(np.int64) if checked.size else \
        np.zeros(0, dtype=np.int64)
    fits = off + out_bytes[checked] <= check_bytes
    checked, off = checked[fits], off[fits]
    out_ptrs[checked] = check_ptr + off
    in_bytes = np.where(dirs == 0, lens, 2 * lens).astype(np.uint64)
    return Workload((tr.arrival_s * 1e9).astype(np.uint64), data_ptrs, lens, dirs, out_ptrs, out_caps, in_bytes,
                    checked, off)


def summarize(w: Workload, lat_ns: np.ndarray, wall_ns: int, rate: float) -> dict:
    lat_us = lat_ns.astype(np.float64) / 1e3
    total = float(np.sum(w.in_bytes))
    return {
        "offered_req_per_s": rate,
        "requests": int(w.arrival_ns.size),
        "input_bytes": int(total),
        "delivered_GBps": round(total / max(wall_ns, 1), 3),
        "p50_us": round(float(np.percentile(lat_us, 50)), 1) if lat_us.size else None,
        "p99_us": round(float(np.percentile(lat_us, 99)), 1) if lat_us.size else None,
        "max_us": round(float(lat_us.max()), 1) if lat_us.size else None,
    }
