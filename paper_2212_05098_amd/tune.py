"""Launch-configuration autotuner.

Single-buffer operations: times each launch configuration the library offers (tile
bytes x tiles per segment x resident workgroups per CU) on synthetic inputs of the
four script profiles and keeps the one with the least total device time.  Batched
call: times every combination of its tunables (longest wave-walked string, tiles per
large-string segment, persistent segment workgroups per CU) on the batched workload
(200,000 strings, log-normal lengths, median 256 B, sigma 2, 8 B .. 4 MiB, mixed
profiles and directions).  Times come from HIP events on the context's stream.  The
choices go to a JSON cache, one entry per (GPU architecture, HIP version, CU count);
Context.load_tuning applies the entry of the GPU it runs on.

Usage:  python -m paper_2212_05098_amd.tune [--size-mib 64] [--out tune_cache.json]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tune_cache.json")

# (tile bytes, tiles per segment) each operation accepts
CANDIDATES = {
    0: [(4096, 2), (4096, 4), (4096, 8), (8192, 2), (8192, 4)],              # UTF-8 -> UTF-16
    1: [(4096, 2), (4096, 4), (4096, 8), (8192, 2), (8192, 4), (8192, 8)],  # UTF-16 -> UTF-8
    2: [(4096, 4), (4096, 8), (8192, 4), (8192, 8), (8192, 16)],            # validate UTF-8
    3: [(4096, 4), (4096, 8), (8192, 4), (8192, 8), (8192, 16)],            # validate UTF-16
    4: [(4096, 8), (8192, 8), (8192, 16)],                                  # length from UTF-8
    5: [(4096, 8), (8192, 8), (8192, 16)],                                  # length from UTF-16
}
# resident workgroups per CU: 0 = as many as fit; larger values than a kernel reaches
# anyway behave like 0
WGS = (0, 1, 2, 3, 4)
# batched call: (longest wave-walked string in units, tiles per large segment, large
# workgroups per CU)
BATCH_CANDIDATES = [(wm, bs, wg) for wm in (4096, 8192, 16384, 32768, 65536) for bs in (2, 4) for wg in (1, 2)]
PROFILES = ("ascii", "latin", "cjk", "emoji")


def device_key() -> str:
    """The cache key of the current GPU: architecture, HIP version, CU count."""
    import torch

    p = torch.cuda.get_device_properties(0)
    return "%s|hip %s|%d CUs" % (getattr(p, "gcnArchName", "unknown"), torch.version.hip, p.multi_processor_count)


def _time(fn, reps):
    import torch

    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(ctx, size_mib: int = 64, reps: int = 5, log=print, batch_strings: int = 200000) -> dict:
    import numpy as np
    import torch

    import paper_2212_05098_amd as utfx
    from paper_2212_05098_amd import synth

    n = size_mib << 20
    res = utfx.result_tensor(1)
    inputs = []
    for prof in PROFILES:
        u8 = torch.from_numpy(synth.config_buffer(prof, 0, n, config=2)).cuda()
        u16 = torch.from_numpy(synth.config_buffer(prof, 1, n, config=2).view(np.int16)).cuda()
        inputs.append((prof, u8, u16))
    out16 = torch.empty(n, dtype=torch.int16, device="cuda")
    out8 = torch.empty(3 * (n // 2), dtype=torch.uint8, device="cuda")
    calls = {
        0: lambda u8, u16: ctx.utf8_to_utf16le_async(u8, out16, res),
        1: lambda u8, u16: ctx.utf16le_to_utf8_async(u16, out8, res),
        2: lambda u8, u16: ctx.validate_utf8_async(u8, res),
        3: lambda u8, u16: ctx.validate_utf16le_async(u16, res),
        4: lambda u8, u16: ctx.utf16_length_from_utf8_async(u8, res),
        5: lambda u8, u16: ctx.utf8_length_from_utf16le_async(u16, res),
    }
    choice = {}
    for op, cands in CANDIDATES.items():
        best = None
        for tile, seg in cands:
            for wgs in WGS:
                cfg = (tile, seg, wgs)
                ctx.set_tuning(op, *cfg)
                ms = sum(_time(lambda: calls[op](u8, u16), reps) for _, u8, u16 in inputs)
                log("op %d %-16s %.4f ms (4 profiles x %d MiB)" % (op, cfg, ms, size_mib))
                if best is None or ms < best[0]:
                    best = (ms, cfg)
        ctx.set_tuning(op, *best[1])
        choice[op] = list(best[1])
    del inputs, out16, out8
    torch.cuda.empty_cache()
    batch = tune_batch(ctx, batch_strings, reps, log) if batch_strings else None
    return {"key": device_key(), "device": torch.cuda.get_device_name(0), "size_mib": size_mib,
            "ops": {str(k): v for k, v in choice.items()}, "batch": batch,
            "batch_strings": batch_strings}


def tune_batch(ctx, n_strings: int, reps: int, log=print):
    """Best (wave_max_units, large_tiles_per_segment, large_wgs_per_cu) of the batched
    call on the batched workload's distribution."""
    import numpy as np
    import torch

    import paper_2212_05098_amd as utfx
    from paper_2212_05098_amd import synth

    b = synth.make_batch(n_strings, seed_key=(0, 4), median=256, sigma=2.0, hi=4 << 20, err_frac=0.005)
    caps, out_off, out_bytes = synth.batch_output_layout(b)
    d_in = torch.from_numpy(b.arena).cuda()
    d_out = torch.empty(out_bytes, dtype=torch.uint8, device="cuda")
    items = utfx.pack_items(b.in_off, b.in_len, out_off, caps, b.direction)
    res = utfx.result_tensor(n_strings)
    total = int(np.sum(b.in_len))
    best = None
    for cfg in BATCH_CANDIDATES:
        ctx.set_batch_tuning(*cfg)
        ms = _time(lambda: ctx.batch_run(d_in, d_out, items, n_strings, total, res), reps)
        log("batch %-20s %.4f ms (%d strings)" % (cfg, ms, n_strings))
        if best is None or ms < best[0]:
            best = (ms, cfg)
    ctx.set_batch_tuning(*best[1])
    return list(best[1])


def save(entry: dict, path: str = DEFAULT_CACHE):
    """Adds (or replaces) the entry of its device key in the cache file."""
    cache = {"entries": {}}
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f)
        if isinstance(old.get("entries"), dict):
            cache = old
    cache["entries"][entry["key"]] = entry
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def load(path: str = DEFAULT_CACHE, key: str = None):
    """The cache entry of the current GPU (or of `key`), or None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        cache = json.load(f)
    entries = cache.get("entries")
    if not isinstance(entries, dict):
        return None
    return entries.get(key if key is not None else device_key())


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--size-mib", type=int, default=64)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--batch-strings", type=int, default=200000, help="0 = skip the batched call")
    a = ap.parse_args(argv)
    import torch

    sys.path.insert(0, os.path.dirname(HERE))
    import paper_2212_05098_amd as utfx

    torch.cuda.set_device(0)
    t0 = time.time()
    with utfx.Context() as ctx:
        entry = tune(ctx, a.size_mib, a.reps, log=lambda m: print(m, flush=True), batch_strings=a.batch_strings)
    save(entry, a.out)
    print("wrote %s in %.1f s: %s / batch %s" % (a.out, time.time() - t0, entry["ops"], entry["batch"]), flush=True)


if __name__ == "__main__":
    main()
