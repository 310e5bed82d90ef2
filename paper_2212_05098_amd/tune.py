"""Launch-configuration autotuner.

For every single-buffer operation it times each launch configuration the library
offers (tile bytes x tiles per segment) on synthetic inputs of the four script
profiles, keeps the one with the least
total device time, and writes the choice to a JSON cache that Context.load_tuning
applies.  Times come from HIP events on the context's stream.

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
PROFILES = ("ascii", "latin", "cjk", "emoji")


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


def tune(ctx, size_mib: int = 64, reps: int = 5, log=print) -> dict:
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
        for cfg in cands:
            ctx.set_tuning(op, *cfg)
            ms = sum(_time(lambda: calls[op](u8, u16), reps) for _, u8, u16 in inputs)
            log("op %d %-12s %.4f ms (4 profiles x %d MiB)" % (op, cfg, ms, size_mib))
            if best is None or ms < best[0]:
                best = (ms, cfg)
        ctx.set_tuning(op, *best[1])
        choice[op] = [best[1][0], best[1][1], ctx.get_tuning(op)[2]]
    return {"device": torch.cuda.get_device_name(0), "size_mib": size_mib, "ops": {str(k): v for k, v in choice.items()}}


def save(cache: dict, path: str = DEFAULT_CACHE):
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def load(path: str = DEFAULT_CACHE):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--size-mib", type=int, default=64)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=DEFAULT_CACHE)
    a = ap.parse_args(argv)
    import torch

    sys.path.insert(0, os.path.dirname(HERE))
    import paper_2212_05098_amd as utfx

    torch.cuda.set_device(0)
    t0 = time.time()
    with utfx.Context() as ctx:
        cache = tune(ctx, a.size_mib, a.reps, log=lambda m: print(m, flush=True))
    save(cache, a.out)
    print("wrote %s in %.1f s: %s" % (a.out, time.time() - t0, cache["ops"]), flush=True)


if __name__ == "__main__":
    main()
