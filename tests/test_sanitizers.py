"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU:

* the oracle (utf_oracle.c and its timing harness) built with -fsanitize=address,
  undefined and loaded in place of the normal build, while the oracle pins and the
  stream-rule test run in a child interpreter (the ASan runtime preloaded first);
* the server's policy harness (serve_policy_harness.cpp, the packing and scheduling
  header the server uses) built and run with the same sanitizers.

A report of either sanitizer fails the run (halt_on_error, no recovery)."""
import os
import shutil
import subprocess
import sys

import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2212_05098_amd", "csrc")


def _runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_pins_under_asan_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if shutil.which("gcc") is None or asan is None:
        pytest.skip("no gcc AddressSanitizer runtime")
    lib = O.build(sanitize=True, lib_path=str(tmp_path / "liboracle_san.so"))
    env = dict(os.environ)
    env["UTFX_ORACLE_LIB"] = lib
    env["LD_PRELOAD"] = asan + ((":" + env["LD_PRELOAD"]) if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_oracle_pins.py"), os.path.join(HERE, "test_stream_rule.py")],
                       capture_output=True, text=True, timeout=900, env=env, cwd=ROOT)
    out = p.stdout + p.stderr
    assert p.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]


def test_serve_policy_harness_under_asan_ubsan(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no C++ compiler")
    exe = tmp_path / "harness_san"
    subprocess.check_call([cxx, "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-Werror",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           "-I", CSRC, os.path.join(HERE, "serve_policy_harness.cpp"), "-o", str(exe)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    p = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert p.returncode == 0, p.stdout + p.stderr
    lines = p.stdout.strip().splitlines()
    assert len(lines) == 4 and all(l.startswith("ok ") for l in lines), p.stdout
