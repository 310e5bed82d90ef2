"""Host logic of the rocprofv3 summaries (CPU): the kernel-trace table and its per-input
split, the traffic calibration against a copy kernel, and that a traffic summary taken
from other kernel sources is not used."""
import csv
import os

from paper_2212_05098_amd import profsum


def _write(path, fields, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_stats_table_and_split(tmp_path):
    rows, t = [], 0
    for i in range(8):  # k_u8_to_u16 on inputs a, b alternating: 100 and 300 ns
        d = 100 if i % 2 == 0 else 300
        rows.append({"Kernel_Name": "void utfx_dev::k_u8_to_u16<512, 4>(Launch)", "Start_Timestamp": t,
                     "End_Timestamp": t + d})
        t += 1000
    rows.append({"Kernel_Name": "k_other", "Start_Timestamp": t, "End_Timestamp": t + 400})
    _write(str(tmp_path / "s" / "run_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    text = profsum.stats_text(str(tmp_path / "s"), "cmd", cycle=["a", "b"])
    lines = [l for l in text.splitlines() if not l.startswith("#")]
    main = [l for l in lines if l.startswith("void k_u8_to_u16<512, 4>(Launch) ") and "[" not in l][0].split()
    assert main[-5:] == ["8", "0.20", "0.10", "0.30", "80.00"]  # 1600 of 2000 ns
    a = [l for l in lines if "[a]" in l][0].split()
    b = [l for l in lines if "[b]" in l][0].split()
    assert a[-5:-1] == ["4", "0.10", "0.10", "0.10"] and b[-5:-1] == ["4", "0.30", "0.30", "0.30"]
    assert "# kernel sources: %s" % profsum.source_hash() in text


def test_traffic_calibration_and_staleness(tmp_path):
    fields = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    copy = profsum.COPY_KERNEL
    fetch = [{"Kernel_Name": copy, "Grid_Size": 1 << 20, "Counter_Name": "FETCH_SIZE", "Counter_Value": 131072.0},
             {"Kernel_Name": copy, "Grid_Size": 64, "Counter_Name": "FETCH_SIZE", "Counter_Value": 1.0},
             {"Kernel_Name": "k_u8_to_u16<512, 4>", "Grid_Size": 8192, "Counter_Name": "FETCH_SIZE",
              "Counter_Value": 65536.0}]
    write = [{"Kernel_Name": copy, "Grid_Size": 1 << 20, "Counter_Name": "WRITE_SIZE", "Counter_Value": 262144.0},
             {"Kernel_Name": "k_u8_to_u16<512, 4>", "Grid_Size": 8192, "Counter_Name": "WRITE_SIZE",
              "Counter_Value": 1024.0}]
    _write(str(tmp_path / "f" / "run_counter_collection.csv"), fields, fetch)
    _write(str(tmp_path / "w" / "run_counter_collection.csv"), fields, write)
    text = profsum.traffic_text(str(tmp_path / "f"), str(tmp_path / "w"), "k_u8_to_u16", "case x", 256 << 20,
                                "cf", "cw")
    kv = dict(l.split(": ", 1) for l in text.splitlines() if ": " in l and not l.startswith("#"))
    # a 256 MiB copy reads 131072 KiB (factor 2) and writes 262144 KiB (factor 1)
    assert kv["fetch_factor"] == "2.0000" and kv["write_factor"] == "1.0000"
    assert int(kv["read_bytes_per_launch"]) == 65536 * 1024 * 2 and int(kv["write_bytes_per_launch"]) == 1024 * 1024
    p = tmp_path / "t.txt"
    p.write_text(text)
    assert profsum.read_traffic(str(p), "k_u8_to_u16", "case x") == 65536 * 2048 + 1024 * 1024
    assert profsum.read_traffic(str(p), "k_u16_to_u8", "case x") is None
    p.write_text(text.replace("kernel_sources: %s" % profsum.source_hash(), "kernel_sources: 0000000000000000"))
    assert profsum.read_traffic(str(p), "k_u8_to_u16", "case x") is None


def test_counters_per_input_and_rates(tmp_path):
    fields = ["Kernel_Name", "Dispatch_Id", "Counter_Name", "Counter_Value"]
    rows = []
    for i in range(1, 9):  # dispatches alternate between inputs a (odd) and b (even)
        a = i % 2 == 1
        clk = 24000 if a else 48000  # 10 us and 20 us at 2.4 GHz
        vals = {"GRBM_GUI_ACTIVE": 8 * clk, "SQ_INSTS_VALU": 1024 * (276 if a else 474),
                "SQ_WAIT_ANY": 256 * clk * (0.5 if a else 0.25)}
        for c, v in vals.items():
            rows.append({"Kernel_Name": "void utfx_dev::k_u8_to_u16<512, 4>(Launch)", "Dispatch_Id": i,
                         "Counter_Name": c, "Counter_Value": float(v)})
    rows.append({"Kernel_Name": "k_other", "Dispatch_Id": 9, "Counter_Name": "SQ_INSTS_VALU",
                 "Counter_Value": 1.0})
    _write(str(tmp_path / "c" / "run_counter_collection.csv"), fields, rows)
    text = profsum.counters_text(str(tmp_path / "c"), "cmd", ["a", "b"], input_kib=1024.0)
    lines = text.splitlines()
    assert "# kernel sources: %s" % profsum.source_hash() in text and "k_other" not in text
    ia = lines.index("void k_u8_to_u16<512, 4> [a]: 4 launches, 10.0 us at 2.4 GHz")
    ib = lines.index("void k_u8_to_u16<512, 4> [b]: 4 launches, 20.0 us at 2.4 GHz")
    a = {l.split()[0]: l.split()[2:] for l in lines[ia + 1:ib]}
    b = {l.split()[0]: l.split()[2:] for l in lines[ib + 1:]}
    # instructions per KiB of input and per CU per clock (1024 * 276 / (256 * 24000))
    assert a == {"SQ_INSTS_VALU": ["276.0", "/KiB", "0.046", "/CU/clk"], "SQ_WAIT_ANY": ["0.500", "/CU/clk"]}
    assert b == {"SQ_INSTS_VALU": ["474.0", "/KiB", "0.040", "/CU/clk"], "SQ_WAIT_ANY": ["0.250", "/CU/clk"]}
    # another kernel chosen by name
    other = profsum.counters_text(str(tmp_path / "c"), "cmd", ["x"], input_kib=1.0, kernels=("k_other",))
    assert "k_other [x]: 1 launches" in other and "k_u8_to_u16" not in other.split("\n", 1)[1]


def test_code_text_ignores_comments_and_layout():
    a = "int f(int x) {  // the length\n  return x + 1; /* one more\n word */\n}\n"
    b = "int f(int x) {\n  // a longer comment\n  // over two lines\n  return x   +   1;\n}"
    c = "int f(int x) { return x + 2; }"
    assert profsum.code_text(a) == profsum.code_text(b) == "int f(int x) { return x + 1; }"
    assert profsum.code_text(c) != profsum.code_text(a)
