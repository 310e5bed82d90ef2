"""Benchmark: validating transcode input GB/s on one MI355X.

Workload (one step): four 256 MiB buffers, one per synthetic script profile
(ASCII-heavy, Latin/Cyrillic/Arabic, CJK, emoji), each transcoded in both directions
with full validation (8 calls, 2 GiB of input).  Inputs are resident in HBM before
the timed region; each (profile, direction) rotates over several device copies so
that no call finds its input in the 256 MB Infinity Cache.

Prints ONE JSON line (rank 0).  `value` = input bytes of the step / step time, the
steps timed with nothing but the calls on the stream.  The same steps then run again
with events per call for the per-call and per-kernel figures: `roofline` describes the
dominant kernel (the transcode kernel with the most device time in the step, over its
four launches, one per profile): algorithmic bytes per launch (input + output,
averaged over those launches) / its average launch duration measured with HIP events
on the launch stream, against the 8 TB/s HBM peak.  `cpu_baseline` times the scalar oracle
on a bounded sample of the same inputs on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MIB = 1 << 20


def log(msg):
    sys.stderr.write("[bench] %s\n" % msg)
    sys.stderr.flush()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size-mib", type=int, default=256, help="bytes per buffer (MiB)")
    ap.add_argument("--rotate", type=int, default=3, help="device copies per input")
    ap.add_argument("--streams", type=int, default=1,
                    help="contexts, each on its own stream, that the timed steps' calls alternate over")
    ap.add_argument("--cpu-sample-mib", type=int, default=128, help="oracle sample per C2 case (MiB)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profiles", default="ascii,latin,cjk,emoji")
    ap.add_argument("--u8", default="", help="UTF-8 -> UTF-16 launch: tile_bytes,tiles_per_segment")
    ap.add_argument("--u16", default="", help="UTF-16 -> UTF-8 launch: tile_bytes,tiles_per_segment")
    ap.add_argument("--batch-strings", type=int, default=200000, help="strings in the batched workload (0 = skip)")
    ap.add_argument("--batch-reps", type=int, default=10)
    ap.add_argument("--single-sample", type=int, default=20000,
                    help="strings of the batch run with one launch each, for the comparison")
    ap.add_argument("--serve-rates", default="20000,50000,100000,200000,500000",
                    help="offered request rates of the serving runs (empty = skip)")
    ap.add_argument("--serve-seconds", type=float, default=5.0, help="trace length per offered rate (s)")
    ap.add_argument("--serve-inflight", type=int, default=3, help="server steps in flight")
    ap.add_argument("--small-calls", type=int, default=200, help="64 KiB synchronous calls timed (0 = skip)")
    ap.add_argument("--run-mib", type=int, default=64, help="run-structured buffers per profile (MiB, 0 = skip)")
    ap.add_argument("--stream-chunks", default="1,16",
                    help="chunk sizes (MiB) of the stream runs over one mixed buffer (empty = skip)")
    ap.add_argument("--stream-mib", type=int, default=256, help="stream length (MiB)")
    ap.add_argument("--utf32-mib", type=int, default=256, help="UTF-32 runs: input MiB per direction (0 = skip)")
    ap.add_argument("--no-tune-cache", action="store_true", help="ignore the tuning cache")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run plain 256 MiB device copies (counter calibration for rocprofv3 --pmc)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2212_05098_amd as utfx
    from paper_2212_05098_amd import synth

    torch.cuda.set_device(0)
    ctx = utfx.Context()
    # further contexts on streams of their own (default priority) for --streams
    ctxs = [ctx] + [utfx.Context(stream=torch.cuda.Stream()) for _ in range(max(args.streams, 1) - 1)]
    for c in ctxs:
        tuned = False if args.no_tune_cache else c.load_tuning()
        for op, spec in ((utfx.OP_UTF8_TO_UTF16, args.u8), (utfx.OP_UTF16_TO_UTF8, args.u16)):
            if spec:
                t, sg = (int(v) for v in spec.split(","))
                c.set_tuning(op, t, sg)
    nbytes = args.size_mib * MIB
    profiles = args.profiles.split(",")
    cases = []  # (profile, direction, host_input, [device copies], device_output, in_bytes, out_bytes)
    for prof in profiles:
        for d in (synth.DIR_8TO16, synth.DIR_16TO8):
            t0 = time.time()
            host = synth.config_buffer(prof, d, nbytes, config=2)
            src = torch.from_numpy(host.view(np.uint8).copy()).cuda()
            copies = [src] + [src.clone() for _ in range(args.rotate - 1)]
            if d == synth.DIR_8TO16:
                out = torch.empty(nbytes, dtype=torch.int16, device="cuda")  # n words
            else:
                copies = [c.view(torch.int16) for c in copies]
                out = torch.empty(3 * (nbytes // 2), dtype=torch.uint8, device="cuda")
            cases.append([prof, d, host, copies, out, nbytes, 0])
            log("generated %s dir=%d in %.1fs" % (prof, d, time.time() - t0))
    res = utfx.result_tensor(len(cases) * 2)

    def call(i, rot, c=ctx):
        prof, d, host, copies, out, nb, _ = cases[i]
        src = copies[rot % len(copies)]
        r = res[24 * i:24 * i + 24]
        if d == synth.DIR_8TO16:
            st = c.utf8_to_utf16le_async(src, out, r)
        else:
            st = c.utf16le_to_utf8_async(src, out, r)
        if st != utfx.OK:
            raise RuntimeError("launch failed: %d %s" % (st, c.last_error()))

    # correctness of the timed configuration (results only; parity tests cover bytes)
    for i in range(len(cases)):
        call(i, 0)
    torch.cuda.synchronize()
    rs = utfx.results_from_tensor(res)
    for i, c in enumerate(cases):
        if rs[i].status != utfx.OK:
            raise RuntimeError("case %s/%d failed: %r" % (c[0], c[1], rs[i]))
        c[6] = rs[i].count * (2 if c[1] == synth.DIR_8TO16 else 1)
        log("case %s dir=%d in=%d out=%d" % (c[0], c[1], c[5], c[6]))

    stream = torch.cuda.current_stream()
    for w in range(args.warmup):
        for i in range(len(cases)):
            call(i, w, ctxs[i % len(ctxs)])
    torch.cuda.synchronize()

    def evpair():
        return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    # the timed steps: the calls alone, back to back on the stream (with --streams, call i
    # on context i mod streams, so that a call's finalisation and last workgroups overlap
    # the next call)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        for i in range(len(cases)):
            call(i, s + 1, ctxs[i % len(ctxs)])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_s = (t1 - t0) / args.steps
    rs = utfx.results_from_tensor(res)
    assert all(r.status == utfx.OK for r in rs[: len(cases)])

    # the same steps again with events per call: around the whole call (main kernel +
    # finalisation) on the stream, and kernel-only events that the library records
    # immediately before and after the main kernel (hipExtLaunchKernel)
    ev = [[evpair() for _ in cases] for _ in range(args.steps)]
    kev = [[evpair() for _ in cases] for _ in range(args.steps)]
    for row in kev:
        for a_, b_ in row:
            a_.record(stream)
            b_.record(stream)
    torch.cuda.synchronize()
    for s in range(args.steps):
        for i in range(len(cases)):
            ev[s][i][0].record(stream)
            ctx.set_kernel_events(*kev[s][i])
            call(i, s + 1)
            ev[s][i][1].record(stream)
    torch.cuda.synchronize()
    ctx.set_kernel_events(None, None)
    rs = utfx.results_from_tensor(res)
    assert all(r.status == utfx.OK for r in rs[: len(cases)])
    in_bytes = sum(c[5] for c in cases)
    per_case = []
    for i, c in enumerate(cases):
        ms = [ev[s][i][0].elapsed_time(ev[s][i][1]) for s in range(args.steps)]
        kms = [kev[s][i][0].elapsed_time(kev[s][i][1]) for s in range(args.steps)]
        avg, kavg = sum(ms) / len(ms), sum(kms) / len(kms)
        per_case.append({
            "profile": c[0], "dir": "utf8->utf16le" if c[1] == 0 else "utf16le->utf8",
            "kernel": "k_u8_to_u16" if c[1] == 0 else "k_u16_to_u8",
            "in_bytes": c[5], "out_bytes": c[6],
            "kernel_ms_avg": round(kavg, 4), "kernel_ms_min": round(min(kms), 4),
            "call_ms_avg": round(avg, 4),
            "in_GBps": round(c[5] / (kavg * 1e6), 1),
            "hbm_frac": round((c[5] + c[6]) / (kavg * 1e6) / HBM_PEAK_GBS, 4),
        })
    # per transcode kernel (one launch per profile): algorithmic bytes per launch and
    # kernel-only duration per launch, both averaged over its launches
    kernels = {}
    for d in (synth.DIR_8TO16, synth.DIR_16TO8):
        pcs = [pc for pc, c in zip(per_case, cases) if c[1] == d]
        if not pcs:
            continue
        launch_ms = sum(pc["kernel_ms_avg"] for pc in pcs) / len(pcs)
        launch_bytes = sum(pc["in_bytes"] + pc["out_bytes"] for pc in pcs) / len(pcs)
        name = pcs[0]["kernel"]
        kernels[name] = {
            "dir": d, "total_ms": sum(pc["kernel_ms_avg"] for pc in pcs), "launch_ms": launch_ms,
            "launch_bytes": launch_bytes, "achieved": launch_bytes / (launch_ms * 1e6),
            "frac_by_profile": {pc["profile"]: pc["hbm_frac"] for pc in pcs},
        }
    kernel = max(kernels, key=lambda k: kernels[k]["total_ms"])
    dom = kernels[kernel]
    achieved = dom["achieved"]
    case_name = "%s, one launch per profile (%s)" % ("utf8->utf16le" if dom["dir"] == synth.DIR_8TO16 else
                                                     "utf16le->utf8", ",".join(profiles))
    for pc in per_case:
        log("%-6s %-14s kernel %8.4f ms (call %8.4f)  in %7.1f GB/s  hbm %.3f" % (
            pc["profile"], pc["dir"], pc["kernel_ms_avg"], pc["call_ms_avg"], pc["in_GBps"], pc["hbm_frac"]))

    # practical ceiling: a plain device-to-device copy of one input buffer
    csrc = cases[0][3][0].view(torch.uint8)
    cdst = torch.empty_like(csrc)
    for _ in range(2):
        cdst.copy_(csrc)
    ce0, ce1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ce0.record(stream)
    for _ in range(5):
        cdst.copy_(csrc)
    ce1.record(stream)
    torch.cuda.synchronize()
    copy_ms = ce0.elapsed_time(ce1) / 5
    copy_gbps = 2 * csrc.numel() / (copy_ms * 1e6)
    if args.copy_probe:
        for _ in range(2):
            cdst.copy_(csrc)
        torch.cuda.synchronize()
    del cdst
    log("device copy %d MiB: %.3f ms = %.1f GB/s (read + write)" % (csrc.numel() // MIB, copy_ms, copy_gbps))

    from paper_2212_05098_amd import profsum

    tpath = os.path.join(ROOT, "profiles", "hbm_traffic_%s_%dMiB.txt" % (kernel, args.size_mib))
    traffic = profsum.read_traffic(tpath, kernel, case_name)
    # the same kernel's timed launches under rocprofv3 (the committed summary, used while
    # its kernel sources match the library's)
    rp_us = profsum.read_timed_us(os.path.join(ROOT, "profiles", "kernel_trace_transcode_4profiles_%dMiB.txt" %
                                               args.size_mib), kernel)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(cases, args.cpu_sample_mib, log)

    small = run_small(ctx, log, args.small_calls) if args.small_calls else None
    runs = run_structured(ctx, log, args.run_mib) if args.run_mib else None
    streamed = run_stream(ctx, log, args.stream_mib, args.stream_chunks) if args.stream_chunks else None
    utf32 = run_utf32(ctx, log, args.utf32_mib) if args.utf32_mib else None
    batch = run_batch(args, ctx, log) if args.batch_strings else None
    serving = run_serving(args, log) if args.serve_rates else None

    out = {
        "metric": "validated transcode input GB/s (% HBM peak); batched p50/p99 latency at load",
        "value": round(in_bytes / step_s / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8/u16 (integer, bit-exact)",
        "data": "synthetic",
        "config": {"workload": "four %d MiB buffers (ascii, latin, cjk, emoji profiles), each transcoded "
                               "UTF-8->UTF-16LE and UTF-16LE->UTF-8 with validation" % args.size_mib,
                   "buffers": len(cases), "bytes_per_buffer": nbytes, "rotate": args.rotate,
                   "streams": len(ctxs),
                   "tuning": {"utf8->utf16le": list(ctx.get_tuning(0)), "utf16le->utf8": list(ctx.get_tuning(1)),
                              "source": "tune_cache.json" if tuned else "defaults"}},
        "roofline": {"bound": "hbm", "kernel": kernel, "case": case_name,
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "algorithmic_bytes": int(dom["launch_bytes"]), "ms_avg": round(dom["launch_ms"], 4),
                     "timing": "kernel-only HIP events around each launch of the kernel (hipExtLaunchKernel)",
                     "frac_by_profile": dom["frac_by_profile"],
                     "traffic": traffic,
                     "rocprof_ms_avg": round(rp_us / 1e3, 4) if rp_us else None,
                     "rocprof_frac": round(dom["launch_bytes"] / (rp_us * 1e3) / HBM_PEAK_GBS, 4) if rp_us else None,
                     "other_kernels": {k: {"achieved": round(v["achieved"], 1),
                                           "frac": round(v["achieved"] / HBM_PEAK_GBS, 4),
                                           "ms_avg": round(v["launch_ms"], 4),
                                           "algorithmic_bytes": int(v["launch_bytes"]),
                                           "frac_by_profile": v["frac_by_profile"]}
                                       for k, v in kernels.items() if k != kernel}},
        "device_copy_GBps": round(copy_gbps, 1),
        "cpu_baseline": cpu,
        "per_case": per_case,
        "small_64KiB": small,
        "run_structured": runs,
        "stream": streamed,
        "utf32": utf32,
        "batched": batch,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)
    for c in ctxs:
        c.close()


def cpu_baseline(cases, sample_mib, log):
    """The oracle timed on this host by its C harness (steady clock inside C, threads
    pinned to the CPUs of the affinity mask, fastest of 3 repetitions after a warm-up,
    the input cut at character boundaries for several threads): on a bounded sample of
    the C2 buffers with 1 thread and with every CPU of the affinity mask, plus the 64 KiB
    buffer (C1), a validation-stress sample (C3) and the batch (C4, in run_batch).  The
    all-CPU result of every sample must equal the 1-thread result."""
    import numpy as np

    import oracle as O
    from paper_2212_05098_amd import synth

    n_cpu = len(os.sched_getaffinity(0))
    sample = sample_mib * MIB
    t1_s = tn_s = 0.0
    nbytes = 0
    used = 1
    for c in cases:
        host = c[2]
        if c[1] == synth.DIR_8TO16:
            part = host[:sample]
            if part.size < host.size:  # cut before the last character that starts in the sample
                lead = part.size - 1
                while lead > 0 and (int(part[lead]) & 0xC0) == 0x80:
                    lead -= 1
                part = part[:lead]
            op, nb = O.TIME_U8_TO_U16, part.size
        else:
            part = host[: sample // 2]
            if part.size and 0xD800 <= part[-1] < 0xDC00:
                part = part[:-1]
            op, nb = O.TIME_U16_TO_U8, 2 * part.size
        one = O.time_buffer(op, part, threads=1, reps=3)
        alln = O.time_buffer(op, part, threads=0, reps=3)
        assert tuple(alln.result) == tuple(one.result), (c[0], c[1], alln.result, one.result)
        assert alln.result.status == 0
        t1_s += one.seconds
        tn_s += alln.seconds
        nbytes += nb
        used = alln.threads
    out = {"value": round(nbytes / tn_s / 1e9, 3), "unit": "GB/s", "cores": used, "kind": "oracle",
           "sample": "first %d MiB of each of the %d C2 (profile, direction) buffers, cut at a character "
                     "boundary; C harness, steady clock, fastest of 3 after a warm-up; %d pinned threads "
                     "(every CPU of the affinity mask), input split at character boundaries" %
                     (sample_mib, len(cases), used),
           "single_thread": {"value": round(nbytes / t1_s / 1e9, 3), "unit": "GB/s", "cores": 1},
           "affinity_cpus": n_cpu}
    log("oracle C2 sample: %.3f GB/s on 1 thread, %.3f GB/s on %d threads" %
        (out["single_thread"]["value"], out["value"], used))
    # C1: the 64 KiB buffer, UTF-8 -> UTF-16LE and back
    d1 = synth.config1_buffer()
    a = O.time_buffer(O.TIME_U8_TO_U16, d1, threads=1, reps=20)
    w = a.out
    b = O.time_buffer(O.TIME_U16_TO_U8, w, threads=1, reps=20)
    out["c1_64KiB"] = {"utf8_to_utf16le_us": round(a.seconds * 1e6, 1), "utf16le_to_utf8_us": round(b.seconds * 1e6, 1),
                       "cores": 1}
    # C3: validation stress samples at the 1e-3 rate, transcode and validate, both directions
    st = {}
    rng = synth.rng_for(0, 3, 1)
    inj8 = synth.inject_utf8("cjk", 32 * MIB, 1e-3, rng)
    inj16 = synth.inject_utf16("mixed4", 16 * MIB, 1e-3, rng)
    for name, op, data in (("utf8->utf16le", O.TIME_U8_TO_U16, inj8.data), ("validate utf8", O.TIME_VALIDATE_U8, inj8.data),
                           ("utf16le->utf8", O.TIME_U16_TO_U8, inj16.data),
                           ("validate utf16le", O.TIME_VALIDATE_U16, inj16.data)):
        one = O.time_buffer(op, data, threads=1, reps=3)
        alln = O.time_buffer(op, data, threads=0, reps=3)
        assert tuple(alln.result) == tuple(one.result) and one.result.status != 0
        st[name] = {"ms_to_verdict_1": round(one.seconds * 1e3, 4), "ms_to_verdict_all": round(alln.seconds * 1e3, 4),
                    "first_error": int(one.result.count)}
    out["c3_stress_1e-3"] = {"sample": "32 MiB CJK UTF-8 and 32 MiB mixed UTF-16LE with errors at rate 1e-3; "
                                       "the oracle stops at the first error, so its time is the time to the verdict",
                             "cases": st}
    return out


def run_small(ctx, log, reps=200):
    """The 64 KiB mixed buffer (characters of all four UTF-8 lengths): synchronous
    UTF-8 -> UTF-16LE and back, the latency a caller sees per call (launch, kernels,
    result copy); the round trip is checked to reproduce the input."""
    import numpy as np
    import torch

    import paper_2212_05098_amd as utfx
    from paper_2212_05098_amd import synth

    data = synth.config1_buffer()
    src = torch.from_numpy(data).cuda()
    w = torch.empty(data.size, dtype=torch.int16, device="cuda")
    back = torch.empty(data.size, dtype=torch.uint8, device="cuda")
    r = ctx.utf8_to_utf16le(src, w)
    r2 = ctx.utf16le_to_utf8(w[: r.written], back)
    ok = r.status == utfx.OK and r2.status == utfx.OK and r2.written == data.size and \
        bool(torch.equal(back[: data.size].cpu(), src.cpu()))
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        r = ctx.utf8_to_utf16le(src, w)
        t1 = time.perf_counter()
        ctx.utf16le_to_utf8(w[: r.written], back)
        t2 = time.perf_counter()
        ts.append((t1 - t0, t2 - t1))
    ts = np.array(ts) * 1e6
    out = {"round_trip_ok": ok, "utf8_to_utf16le_us_p50": round(float(np.median(ts[:, 0])), 1),
           "utf16le_to_utf8_us_p50": round(float(np.median(ts[:, 1])), 1), "calls": reps}
    log("64 KiB sync calls: utf8->utf16le %.1f us, utf16le->utf8 %.1f us (p50), round trip %s" %
        (out["utf8_to_utf16le_us_p50"], out["utf16le_to_utf8_us_p50"], "ok" if ok else "MISMATCH"))
    return out


def run_stream(ctx, log, mib, chunk_list, reps=3):
    """One mixed-profile UTF-8 buffer passed as a stream of chunks (each chunk one byte
    longer than a whole number of MiB, so cuts fall inside characters), UTF-8 ->
    UTF-16LE: wall time of the whole stream beside one synchronous call on the buffer;
    the streamed output is checked against the one-call output."""
    import numpy as np
    import torch

    import paper_2212_05098_amd as utfx
    from paper_2212_05098_amd import synth

    data = synth.config_buffer("mixed4", synth.DIR_8TO16, mib << 20, config=2)
    n = data.size
    src = torch.from_numpy(data).cuda()
    whole = torch.empty(n, dtype=torch.int16, device="cuda")
    dst = torch.empty(n, dtype=torch.int16, device="cuda")
    r = ctx.utf8_to_utf16le(src, whole)
    assert r.status == utfx.OK
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.utf8_to_utf16le(src, whole)
        ts.append(time.perf_counter() - t0)
    one = float(np.median(ts))
    out = {"mib": mib, "profile": "mixed4", "dir": "utf8->utf16le", "one_call_ms": round(one * 1e3, 3),
           "runs": []}
    log("stream %d MiB mixed4 utf8->utf16le: one synchronous call %.3f ms" % (mib, one * 1e3))
    for c in [int(x) for x in chunk_list.split(",") if x]:
        chunk = (c << 20) + 1
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = ctx.open_stream(utfx.STREAM_UTF8_TO_UTF16LE)
            pos, calls = 0, 0
            for a in range(0, n, chunk):
                b = min(n, a + chunk)
                rr = st.transcode(src[a:b], dst[pos:pos + st.n_carry + (b - a)], final=b == n)
                pos += rr.written
                calls += 1
            ts.append(time.perf_counter() - t0)
            assert rr.status == utfx.OK and pos == r.written
        ok = bool(torch.equal(dst[:pos], whole[:pos]))
        t = float(np.median(ts))
        out["runs"].append({"chunk_bytes": chunk, "calls": calls, "ms": round(t * 1e3, 3),
                            "in_GBps": round(n / t / 1e9, 1), "us_per_call": round(t / calls * 1e6, 1),
                            "matches_one_call": ok})
        log("stream chunks of %d MiB + 1 B: %d calls, %.3f ms (%.1f GB/s, %.1f us per call), output %s" %
            (c, calls, t * 1e3, n / t / 1e9, t / calls * 1e6, "matches" if ok else "MISMATCH"))
    return out


def run_utf32(ctx, log, mib, reps=5):
    """UTF-32LE: mixed-profile UTF-8 -> UTF-32, and CJK / emoji UTF-32 -> UTF-8,
    UTF-32 -> UTF-16LE and UTF-16LE -> UTF-32 on buffers of `mib` MiB of input, device time per call (HIP events around repeated
    async calls) and HBM bytes (input + output) per second."""
    import numpy as np
    import torch

    import paper_2212_05098_amd as utfx
    from paper_2212_05098_amd import synth

    n = mib << 20
    res = utfx.result_tensor(1)
    out = {"mib": mib, "cases": []}

    def timed(f, src, dst):
        f(src, dst, res)
        torch.cuda.synchronize()
        r = utfx.results_from_tensor(res)[0]
        assert r.status == utfx.OK
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f(src, dst, res)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, r.written

    data = synth.config_buffer("mixed4", synth.DIR_8TO16, n, config=2)
    src = torch.from_numpy(data).cuda()
    dst = torch.empty(n, dtype=torch.int32, device="cuda")
    ms, w = timed(ctx.utf8_to_utf32le_async, src, dst)
    cases = [("mixed4", "utf8->utf32le", n, 4 * w, ms)]
    del src, dst
    for prof in ("cjk", "emoji"):
        units = synth.utf32_buffer(prof, n // 4, synth.rng_for(0, 9, synth.PROFILE_IDS[prof]))
        src = torch.from_numpy(units.view(np.int32)).cuda()
        dst = torch.empty(n, dtype=torch.uint8, device="cuda")
        ms, w = timed(ctx.utf32le_to_utf8_async, src, dst)
        cases.append((prof, "utf32le->utf8", n, w, ms))
        dst = torch.empty(n // 2, dtype=torch.int16, device="cuda")
        ms, w = timed(ctx.utf32le_to_utf16le_async, src, dst)
        cases.append((prof, "utf32le->utf16le", n, 2 * w, ms))
        del src, dst
        words = synth.config_buffer(prof, synth.DIR_16TO8, n, config=2)
        src = torch.from_numpy(words.view(np.int16)).cuda()
        dst = torch.empty(n // 2, dtype=torch.int32, device="cuda")
        ms, w = timed(ctx.utf16le_to_utf32le_async, src, dst)
        cases.append((prof, "utf16le->utf32le", n, 4 * w, ms))
        del src, dst
    torch.cuda.empty_cache()
    for prof, d, nin, nout, ms in cases:
        case = {"profile": prof, "dir": d, "in_bytes": nin, "out_bytes": int(nout), "ms_avg": round(ms, 4),
                "in_GBps": round(nin / (ms * 1e6), 1), "hbm_frac": round((nin + nout) / (ms * 1e6) / HBM_PEAK_GBS, 4)}
        out["cases"].append(case)
        log("utf32 %-6s %-14s %8.3f ms  in %7.1f GB/s  hbm %.3f" % (prof, d, ms, case["in_GBps"], case["hbm_frac"]))
    return out


def run_structured(ctx, log, mib, reps=5):
    """Run-structured text (words in same-script sentences, closer to the paper's lipsum
    files) per profile and direction: device time per call and input GB/s, beside an
    i.i.d. buffer of the same profile and size.  The wave-uniform content classes make
    uniform stretches cheaper."""
    import numpy as np
    import torch

    import paper_2212_05098_amd as utfx
    from paper_2212_05098_amd import synth

    n = mib << 20
    res = utfx.result_tensor(1)
    out = {"mib": mib, "cases": []}

    def timed(host, d):
        if d == synth.DIR_8TO16:
            src = torch.from_numpy(host).cuda()
            dst = torch.empty(n, dtype=torch.int16, device="cuda")
            f = ctx.utf8_to_utf16le_async
        else:
            src = torch.from_numpy(host.view(np.int16)).cuda()
            dst = torch.empty(3 * (n // 2), dtype=torch.uint8, device="cuda")
            f = ctx.utf16le_to_utf8_async
        f(src, dst, res)
        torch.cuda.synchronize()
        assert utfx.results_from_tensor(res)[0].status == utfx.OK
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f(src, dst, res)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    for prof in synth.SCRIPT_PROFILES:
        rng = synth.rng_for(0, 7, synth.PROFILE_IDS[prof])
        for d in (synth.DIR_8TO16, synth.DIR_16TO8):
            run = synth.run_utf8_buffer(prof, n, rng) if d == synth.DIR_8TO16 else synth.run_utf16_buffer(prof, n // 2, rng)
            ms = timed(run, d)
            ms_iid = timed(synth.config_buffer(prof, d, n, config=7), d)
            case = {"profile": prof, "dir": "utf8->utf16le" if d == 0 else "utf16le->utf8", "ms_avg": round(ms, 4),
                    "in_GBps": round(n / (ms * 1e6), 1), "iid_ms_avg": round(ms_iid, 4)}
            out["cases"].append(case)
            log("run-structured %-6s %-14s %8.3f ms  in %7.1f GB/s  (i.i.d. same size %.3f ms)" %
                (prof, case["dir"], ms, case["in_GBps"], ms_iid))
    return out


def run_batch(args, ctx, log):
    """Batched call on many strings (log-normal lengths, median 256 B, sigma 2, 8 B .. 4
    MiB, mixed profiles and directions, 0.5 % with an error): device time per call, and
    the same strings with one launch each (a sample, extrapolated)."""
    import numpy as np
    import torch

    import paper_2212_05098_amd as utfx
    from paper_2212_05098_amd import synth

    t0 = time.time()
    b = synth.make_batch(args.batch_strings, seed_key=(0, 4), median=256, sigma=2.0, hi=4 << 20, err_frac=0.005)
    n = args.batch_strings
    caps = np.where(b.direction == 0, b.in_len, 3 * b.in_len).astype(np.uint64)
    sizes = np.where(b.direction == 0, 2 * caps, caps)
    out_off = np.concatenate([[0], np.cumsum(sizes + 16)[:-1]]).astype(np.uint64)
    out_off += out_off % 2
    d_in = torch.from_numpy(b.arena).cuda()
    d_out = torch.empty(int(out_off[-1] + sizes[-1] + 64), dtype=torch.uint8, device="cuda")
    items = utfx.pack_items(b.in_off, b.in_len, out_off, caps, b.direction)
    res = utfx.result_tensor(n)
    total = int(np.sum(b.in_len))
    in_bytes = int(np.sum(np.where(b.direction == 0, b.in_len, 2 * b.in_len)))
    log("batch: %d strings, %.1f MB generated in %.1fs" % (n, in_bytes / 1e6, time.time() - t0))
    stream = torch.cuda.current_stream()
    for _ in range(2):
        assert ctx.batch_run(d_in, d_out, items, n, total, res) == utfx.OK
    torch.cuda.synchronize()
    rs = utfx.results_from_tensor(res)
    n_err = sum(1 for r in rs if r.status != utfx.OK)
    ms = []
    for _ in range(args.batch_reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        assert ctx.batch_run(d_in, d_out, items, n, total, res) == utfx.OK
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    ms = np.array(ms)
    out_bytes = int(sum(2 * r.written if b.direction[j] == 0 else r.written for j, r in enumerate(rs)))
    # the same call captured into a hipGraph and replayed
    ctx.capture_begin()
    try:
        assert ctx.batch_run(d_in, d_out, items, n, total, res) == utfx.OK
    finally:
        g = ctx.capture_end()
    g.launch()
    torch.cuda.synchronize()
    gms = []
    for _ in range(args.batch_reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.launch()
        e1.record(stream)
        torch.cuda.synchronize()
        gms.append(e0.elapsed_time(e1))
    g.close()
    gms = np.array(gms)
    rs_graph = utfx.results_from_tensor(res)
    # parity of every string's result with the oracle's batched reference, and the
    # oracle timed on the same batch (1 thread, every CPU of the affinity mask)
    oracle_leg = None
    if not args.no_cpu:
        import oracle as O

        items_np = O.items_array(b.in_off, b.in_len, out_off, caps, b.direction)
        o_bytes = int(out_off[-1] + sizes[-1] + 64)
        t1, used1, ores, n_ok = O.time_batch(b.arena, items_np, o_bytes, threads=1, reps=3)
        tn, usedn, ores_n, _ = O.time_batch(b.arena, items_np, o_bytes, threads=0, reps=3)
        got = np.array([(r.status, r.count, r.written) for r in rs_graph], dtype=np.int64)
        want = np.stack([ores["status"].astype(np.int64), ores["count"].astype(np.int64),
                         ores["written"].astype(np.int64)], axis=1)
        mism = int(np.count_nonzero(np.any(got != want, axis=1)))
        assert np.array_equal(ores_n["count"], ores["count"])
        oracle_leg = {"GBps_1": round(in_bytes / t1 / 1e9, 3), "GBps_all": round(in_bytes / tn / 1e9, 3),
                      "cores": usedn, "result_mismatches": mism, "checked": n}
        log("batch oracle: %.3f GB/s on 1 thread, %.3f GB/s on %d; %d of %d results differ from the GPU's" %
            (oracle_leg["GBps_1"], oracle_leg["GBps_all"], usedn, mism, n))
    # one launch per string on a sample (the first k strings), same kernels' results
    k = min(args.single_sample, n)
    one = utfx.result_tensor(1)
    srcs = []
    for i in range(k):
        a, L, o = int(b.in_off[i]), int(b.in_len[i]), int(out_off[i])
        if b.direction[i] == 0:
            srcs.append((0, d_in[a:a + L], d_out[o:o + 2 * int(caps[i])].view(torch.int16)))
        else:
            srcs.append((1, d_in[a:a + 2 * L].view(torch.int16), d_out[o:o + int(caps[i])]))
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for d, src, dst in srcs:
        if d == 0:
            ctx.utf8_to_utf16le_async(src, dst, one)
        else:
            ctx.utf16le_to_utf8_async(src, dst, one)
    torch.cuda.synchronize()
    single_s = time.perf_counter() - ts
    per_string_us = single_s / k * 1e6 if k else float("nan")
    batch_ms = float(np.median(ms))
    log("batch: %.3f ms median per call (%.1f GB/s); one launch per string: %.2f us each" %
        (batch_ms, in_bytes / (batch_ms * 1e6), per_string_us))
    graph_ms = float(np.median(gms))
    log("batch graph replay: %.3f ms median per call (%.1f GB/s)" % (graph_ms, in_bytes / (graph_ms * 1e6)))
    return {"strings": n, "input_bytes": in_bytes, "output_bytes": out_bytes, "errors": n_err,
            "reps": args.batch_reps,
            "ms_p50": round(batch_ms, 4), "ms_p99": round(float(np.percentile(ms, 99)), 4),
            "ms_min": round(float(ms.min()), 4), "GBps": round(in_bytes / (batch_ms * 1e6), 2),
            "hbm_frac": round((in_bytes + out_bytes) / (batch_ms * 1e6) / HBM_PEAK_GBS, 4),
            "graph_ms_p50": round(graph_ms, 4), "graph_ms_p99": round(float(np.percentile(gms, 99)), 4),
            "graph_GBps": round(in_bytes / (graph_ms * 1e6), 2),
            "oracle": oracle_leg,
            "one_launch_per_string_us": round(per_string_us, 2) if k else None, "one_launch_sample": k,
            "speedup_vs_one_launch_per_string": round(per_string_us * n / (batch_ms * 1e3), 1) if k else None}


def check_served(w, res, out_bytes_at, log, label):
    """The served results and outputs of the workload's checked sample against the
    oracle, one request at a time: returns (checked, mismatches).  out_bytes_at(off, n)
    gives n bytes of the sample's output buffer at byte offset off."""
    import ctypes

    import numpy as np

    import oracle as O

    bad = 0
    for idx, off in zip(w.checked.tolist(), w.check_off.tolist()):
        d = int(w.dirs[idx]) & 1
        n = int(w.len_units[idx])
        raw = ctypes.string_at(int(w.data_ptrs[idx]), n * (2 if d else 1)) if n else b""
        if d == 0:
            want, ref = O.utf8_to_utf16le(np.frombuffer(raw, dtype=np.uint8))
            unit = 2
        else:
            want, ref = O.utf16le_to_utf8(np.frombuffer(raw, dtype=np.uint16))
            unit = 1
        r = res[idx]
        ok = (int(r["status"]), int(r["count"]), int(r["written"])) == tuple(want)
        if ok and want.written:
            got = np.frombuffer(out_bytes_at(off, int(want.written) * unit), dtype=ref.dtype)
            ok = np.array_equal(got, ref[: want.written])
        bad += 0 if ok else 1
    if bad:
        log("%s: %d of %d sampled requests differ from the oracle" % (label, bad, w.checked.size))
    return int(w.checked.size), bad


def run_serving(args, log):
    """Continuous-batching server (--serve-inflight steps in flight) on Poisson traces at
    each offered rate: host-resident requests (latency includes PCIe both ways),
    device-resident requests (payload and output in device memory, only results cross
    PCIe), and one launch per request.  Each server first replays an unrecorded 0.2 s
    warm-up trace.  A 1 % sample of each run's requests gets its own output buffer and
    is checked against the oracle."""
    import ctypes

    import numpy as np
    import torch

    import paper_2212_05098_amd as utfx
    from paper_2212_05098_amd import serve

    t0 = time.time()
    pool = serve.PayloadPool(mib_per_pool=32, seed=0)
    # the same payloads in device memory, for the device-resident runs
    dev_pool = {k: t.cuda() for k, t in pool.buf.items()}
    scratch = torch.empty(64 << 20, dtype=torch.uint8, pin_memory=True)
    check = torch.empty(1 << 30, dtype=torch.uint8, pin_memory=True)
    d_scratch = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    d_check = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    log("serving: payload pool in %.1fs" % (time.time() - t0))
    rates = [float(r) for r in args.serve_rates.split(",") if r]
    out = {"server": {"inflight": args.serve_inflight, "arena_in_MiB": 256, "arena_out_MiB": 768,
                      "device_cap_GiB": 32},
           "duration_s": args.serve_seconds, "check_every": 100, "runs": [], "device_resident": [],
           "one_launch_per_request": []}
    srv = utfx.Server(arena_in_bytes=256 << 20, arena_out_bytes=768 << 20, max_items=1 << 18,
                      inflight=args.serve_inflight)

    def warm(server):
        # an unrecorded replay first: the HIP runtime sets up each pinned host buffer
        # the first time a copy uses it (several ms), which would otherwise land in the
        # first measured trace
        w = serve.make_workload(pool, 200000, 0.2, seed=1000, scratch_ptr=scratch.data_ptr(), check_every=50,
                                check_ptr=check.data_ptr(), check_bytes=check.numel())
        server.replay(w.arrival_ns, w.data_ptrs, w.len_units, w.dirs, w.out_ptrs, w.out_caps)
        data, outs, dirs = to_device(w)
        server.replay(w.arrival_ns, data, w.len_units, dirs, outs, w.out_caps)

    def host_reader(off, n):
        return ctypes.string_at(check.data_ptr() + off, n)

    def to_device(w):
        """Device pointers for the same requests: payloads in the device copy of the
        pool, outputs in device buffers (the checked sample at the same offsets)."""
        data = w.data_ptrs.copy()
        for key, t in pool.buf.items():
            lo, hi = t.data_ptr(), t.data_ptr() + t.numel()
            m = (w.data_ptrs >= lo) & (w.data_ptrs < hi)
            data[m] = w.data_ptrs[m] - lo + dev_pool[key].data_ptr()
        outs = np.full(w.out_ptrs.size, d_scratch.data_ptr(), dtype=np.uint64)
        outs[w.checked] = d_check.data_ptr() + w.check_off.astype(np.uint64)
        return data, outs, (w.dirs | utfx.SERVER_DEVICE_BUFFERS).astype(np.uint32)

    def run(server, w, rate, device, label):
        if device:
            data, outs, dirs = to_device(w)
            lat, res, wall = server.replay(w.arrival_ns, data, w.len_units, dirs, outs, w.out_caps)
            host_check = d_check.cpu().numpy()
            reader = lambda off, n: host_check[off:off + n].tobytes()  # noqa: E731
        else:
            lat, res, wall = server.replay(w.arrival_ns, w.data_ptrs, w.len_units, w.dirs, w.out_ptrs, w.out_caps)
            reader = host_reader
        row = serve.summarize(w, lat, wall, rate)
        row["ok"] = int(np.sum(res["status"] == 0))
        if not args.no_cpu:  # the oracle leg: the sampled requests against the oracle
            row["parity_sample"], row["parity_mismatches"] = check_served(w, res, reader, log, label)
            row["parity_sample_ok"] = row["parity_mismatches"] == 0
        else:
            row["parity_sample"], row["parity_mismatches"], row["parity_sample_ok"] = 0, None, None
        log("%s %7.0f req/s: %d requests in %.2f s, p50 %.1f us, p99 %.1f us, %.2f GB/s; sample %d, %s mismatches" %
            (label, rate, row["requests"], w.arrival_ns[-1] / 1e9 if w.arrival_ns.size else 0.0, row["p50_us"],
             row["p99_us"], row["delivered_GBps"], row["parity_sample"], row["parity_mismatches"]))
        return row

    warm(srv)
    for k, rate in enumerate(rates):
        w = serve.make_workload(pool, rate, args.serve_seconds, seed=k, scratch_ptr=scratch.data_ptr(),
                                check_every=100, check_ptr=check.data_ptr(), check_bytes=check.numel())
        out["runs"].append(run(srv, w, rate, False, "serving"))
        out["device_resident"].append(run(srv, w, rate, True, "serving (device-resident)"))
    srv.close()
    # one launch per request (max_items = 1): it cannot keep up with the higher rates,
    # so its traces are cut to at most 100,000 requests (stated per run)
    one = utfx.Server(arena_in_bytes=64 << 20, arena_out_bytes=192 << 20, max_items=1, inflight=2)
    warm(one)
    for k, rate in enumerate(rates):
        dur = min(args.serve_seconds, 100000.0 / rate)
        w = serve.make_workload(pool, rate, dur, seed=k, scratch_ptr=scratch.data_ptr(), check_every=100,
                                check_ptr=check.data_ptr(), check_bytes=check.numel())
        row = run(one, w, rate, False, "one launch per request")
        row["duration_s"] = round(dur, 3)
        out["one_launch_per_request"].append(row)
    one.close()
    return out


if __name__ == "__main__":
    main()
