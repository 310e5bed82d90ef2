"""Summaries of rocprofv3 output for the kernels of this library.

Turns the CSV files of `rocprofv3 --kernel-trace --stats --output-format csv` and of
`rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` into the short text summaries kept
with the sources, and reads the HBM-traffic summary back for bench.py.

HBM traffic of a kernel = FETCH_SIZE and WRITE_SIZE (KiB per dispatch, averaged over
its dispatches), each scaled by the factor that maps the same counter onto the known
traffic of a plain device-to-device copy of `copy_bytes` measured in the same run
(the copy reads and writes copy_bytes each).  The summary records a hash of the
kernel sources; bench.py reports the traffic only while the sources still match.

Usage:
  python -m paper_2212_05098_amd.profsum stats DIR --cmd "..."             > summary.txt
  python -m paper_2212_05098_amd.profsum traffic FETCH_DIR WRITE_DIR --kernel NAME
         --case "utf8->utf16le, one launch per profile (ascii,latin,cjk,emoji)" --copy-bytes 268435456 --cmd "..." > summary.txt
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ("csrc/utfx.hip", "csrc/utfx_kernels.hpp", "csrc/utfx_device.hpp", "csrc/utfx_transcode.hpp",
           "csrc/utfx_batch.hpp")
COPY_KERNEL = "copyBuffer"


_COMMENT = re.compile(r"//[^\n]*|/\*.*?\*/", re.S)


def code_text(text: str) -> str:
    """C++ source text without its comments and with every run of whitespace reduced to
    one space: what decides the compiled code, so that editing a comment leaves the
    summaries valid.  (The kernel sources hold no comment markers inside string or
    character literals, which this does not parse.)"""
    return " ".join(_COMMENT.sub(" ", text).split())


def source_hash() -> str:
    """Hash of what decides the profiled kernels: their sources' code (comments and
    layout left out), the compiler flags and the tuning cache that picks their launch
    shapes."""
    from . import build as B

    h = hashlib.sha256()
    for rel in SOURCES + ("tune_cache.json",):
        p = os.path.join(HERE, rel)
        if os.path.exists(p):
            with open(p, "rb") as f:
                data = f.read()
            if not rel.endswith(".json"):
                data = code_text(data.decode("utf-8")).encode("utf-8")
            h.update(rel.encode() + b"\0" + data)
    h.update(b"flags\0" + " ".join(B.HIPCC_FLAGS).encode())
    return h.hexdigest()[:16]


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError("no *%s under %s" % (suffix, d))
    return hits[0]


def _short(name: str) -> str:
    name = name.replace("utfx_dev::", "")
    return name[:70]


def stats_text(d: str, cmd: str, cycle=None, timed: int = 0) -> str:
    """Per-kernel dispatch count and durations from a kernel-trace run.  With `cycle`
    (the inputs a kernel is dispatched on, in the order the program cycles through
    them), the main kernels are also split per input by dispatch index; with `timed`,
    also the average over the last `timed` dispatches per input (the launches the
    benchmark times, after its correctness and warm-up passes)."""
    rows = list(csv.DictReader(open(_find(d, "kernel_trace.csv"))))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    per = collections.defaultdict(list)
    for r in rows:
        per[r["Kernel_Name"]].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    tot = sum(sum(v) for v in per.values())
    fmt = "%-70s %6d %12.2f %12.2f %12.2f %6.2f"
    out = ["# rocprofv3 kernel trace summary", "# command: %s" % cmd, "# kernel sources: %s" % source_hash(),
           "%-70s %6s %12s %12s %12s %6s" % ("kernel", "calls", "avg_us", "min_us", "max_us", "pct")]
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        out.append(fmt % (_short(k), len(v), sum(v) / len(v) / 1e3, min(v) / 1e3, max(v) / 1e3,
                          100.0 * sum(v) / tot))
    if cycle:
        out.append("# per input (dispatch i of a kernel ran on input i mod %d)" % len(cycle))
        for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
            if not ("k_u8_to_u16<" in k or "k_u16_to_u8<" in k) or len(v) % len(cycle):
                continue
            for j, name in enumerate(cycle):
                w = v[j::len(cycle)]
                out.append(fmt % ("%s [%s]" % (_short(k)[:52], name), len(w), sum(w) / len(w) / 1e3,
                                  min(w) / 1e3, max(w) / 1e3, 100.0 * sum(w) / tot))
        if timed:
            out.append("# timed launches: the last %d dispatches per input of each main kernel" % timed)
            for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
                if not ("k_u8_to_u16<" in k or "k_u16_to_u8<" in k) or len(v) % len(cycle):
                    continue
                w = [x for j in range(len(cycle)) for x in v[j::len(cycle)][-timed:]]
                out.append(fmt % ("%s [timed]" % _short(k)[:52], len(w), sum(w) / len(w) / 1e3, min(w) / 1e3,
                                  max(w) / 1e3, 100.0 * sum(w) / tot))
    return "\n".join(out) + "\n"


def counters_text(d: str, cmd: str, cycle, input_kib: float, cus: int = 256, xcds: int = 8,
                  kernels=("k_u8_to_u16<", "k_u16_to_u8<")) -> str:
    """Per kernel (names containing one of `kernels`) and input (dispatch i ran on input
    i mod len(cycle)): the average value per launch of every counter of a `--pmc` run,
    SQ_INSTS_* also per KiB of input and per CU per clock, the others per CU per clock;
    the clocks of a launch are GRBM_GUI_ACTIVE over the XCDs (it counts on each of
    them)."""
    rows = list(csv.DictReader(open(_find(d, "counter_collection.csv"))))
    per = collections.OrderedDict()  # (kernel, dispatch) -> {counter: value}
    for r in rows:
        k = r["Kernel_Name"]
        if not any(s in k for s in kernels):
            continue
        per.setdefault((_short(k).split("(")[0], int(r["Dispatch_Id"])), {})[r["Counter_Name"]] = \
            float(r["Counter_Value"])
    out = ["# rocprofv3 counters of %s" % ", ".join(s.rstrip("<(") for s in kernels), "# command: %s" % cmd,
           "# kernel sources: %s" % source_hash(),
           "# per launch: average over the launches of each input; /KiB: per KiB of input; /CU/clk: per CU",
           "# per clock, clocks = GRBM_GUI_ACTIVE / %d XCDs (the SQ cycle counters are as read)" % xcds]
    found = sorted({k for k, _ in per}, key=lambda k: min(i for kk, i in per if kk == k))
    for k in found:
        disp = sorted(i for kk, i in per if kk == k)
        for j, name in enumerate(cycle):
            ds = disp[j::len(cycle)]
            if not ds:
                continue
            names = sorted(per[(k, ds[0])])
            avg = {c: sum(per[(k, i)].get(c, 0.0) for i in ds) / len(ds) for c in names}
            clk = avg.get("GRBM_GUI_ACTIVE", 0.0) / xcds
            parts = ["%s [%s]: %d launches, %.1f us at 2.4 GHz" % (k, name, len(ds), clk / 2400.0)]
            for c in names:
                if c == "GRBM_GUI_ACTIVE":
                    continue
                if c.startswith("SQ_INSTS"):
                    parts.append("  %-24s %14.0f  %10.1f /KiB  %8.3f /CU/clk" %
                                 (c, avg[c], avg[c] / input_kib, avg[c] / (cus * clk) if clk else 0.0))
                elif clk:
                    parts.append("  %-24s %14.0f  %10.3f /CU/clk" % (c, avg[c], avg[c] / (cus * clk)))
            out.extend(parts)
    return "\n".join(out) + "\n"


def _counter(d: str, name: str):
    """Kernel name -> [(grid size, counter value)] per dispatch."""
    rows = list(csv.DictReader(open(_find(d, "counter_collection.csv"))))
    per = collections.defaultdict(list)
    for r in rows:
        if r["Counter_Name"] == name:
            per[r["Kernel_Name"]].append((int(r["Grid_Size"]), float(r["Counter_Value"])))
    return per


def traffic_text(fetch_dir: str, write_dir: str, kernel: str, case: str, copy_bytes: int, cmd_f: str,
                 cmd_w: str) -> str:
    fe = _counter(fetch_dir, "FETCH_SIZE")
    wr = _counter(write_dir, "WRITE_SIZE")

    def pick(per, sub):
        # dispatches of the largest grid only: the copy kernel also serves small copies
        ks = [k for k in per if sub in k]
        if not ks:
            raise KeyError("kernel %r not in counters (have %s)" % (sub, list(per)))
        gv = [gv for k in ks for gv in per[k]]
        gmax = max(g for g, _ in gv)
        vals = [v for g, v in gv if g == gmax]
        return sum(vals) / len(vals), len(vals)

    cf, _ = pick(fe, COPY_KERNEL)
    cw, _ = pick(wr, COPY_KERNEL)
    f_factor = copy_bytes / (cf * 1024.0)
    w_factor = copy_bytes / (cw * 1024.0)
    kf, nf = pick(fe, kernel)
    kw, nw = pick(wr, kernel)
    rd = kf * 1024.0 * f_factor
    wb = kw * 1024.0 * w_factor
    lines = [
        "# HBM traffic of %s (%s), rocprofv3 --pmc" % (kernel, case),
        "# fetch command: %s" % cmd_f,
        "# write command: %s" % cmd_w,
        "kernel: %s" % kernel,
        "case: %s" % case,
        "kernel_sources: %s" % source_hash(),
        "copy_bytes: %d" % copy_bytes,
        "copy_FETCH_SIZE_KiB: %.1f" % cf,
        "copy_WRITE_SIZE_KiB: %.1f" % cw,
        "fetch_factor: %.4f" % f_factor,
        "write_factor: %.4f" % w_factor,
        "kernel_FETCH_SIZE_KiB: %.1f (avg of %d dispatches)" % (kf, nf),
        "kernel_WRITE_SIZE_KiB: %.1f (avg of %d dispatches)" % (kw, nw),
        "read_bytes_per_launch: %d" % round(rd),
        "write_bytes_per_launch: %d" % round(wb),
        "traffic_bytes_per_launch: %d" % round(rd + wb),
    ]
    return "\n".join(lines) + "\n"


def read_traffic(path: str, kernel: str, case: str):
    """Traffic bytes per launch from a summary, or None if absent, for another
    kernel/case, or taken from kernel sources that have changed since."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel") != kernel or kv.get("case") != case or kv.get("kernel_sources") != source_hash():
        return None
    return int(kv["traffic_bytes_per_launch"])


def read_timed_us(path: str, kernel: str):
    """Average duration (us) of the timed launches of a main kernel from a kernel-trace
    summary, or None if absent or taken from kernel sources that have changed since."""
    if not os.path.exists(path):
        return None
    src = None
    for line in open(path):
        if line.startswith("# kernel sources:"):
            src = line.split(":", 1)[1].strip()
        elif kernel + "<" in line and "[timed]" in line:
            if src != source_hash():
                return None
            return float(line.split()[-4])
    return None


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--cmd", required=True)
    s.add_argument("--cycle", default="", help="comma-separated inputs the kernels cycle through")
    s.add_argument("--timed", type=int, default=0, help="last dispatches per input the benchmark times")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("--kernel", required=True)
    t.add_argument("--case", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("--cmd", required=True)
    c.add_argument("--cycle", required=True, help="comma-separated inputs the kernels cycle through")
    c.add_argument("--kernels", default="k_u8_to_u16<,k_u16_to_u8<",
                   help="comma-separated parts of the kernel names to summarise")
    c.add_argument("--input-kib", type=float, required=True, help="input KiB per launch")
    a = ap.parse_args(argv)
    if a.what == "counters":
        sys.stdout.write(counters_text(a.dir, a.cmd, [x for x in a.cycle.split(",") if x], a.input_kib,
                                       kernels=tuple(k for k in a.kernels.split(",") if k)))
    elif a.what == "stats":
        sys.stdout.write(stats_text(a.dir, a.cmd, [c for c in a.cycle.split(",") if c], a.timed))
    else:
        sys.stdout.write(traffic_text(a.fetch_dir, a.write_dir, a.kernel, a.case, a.copy_bytes, a.cmd_fetch,
                                      a.cmd_write))


if __name__ == "__main__":
    main()
