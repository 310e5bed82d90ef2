"""The server's packing and scheduling decisions (utfx_serve_policy.hpp, the header the
server itself uses) under a mock executor on a virtual clock, on the CPU: compiled with
the host compiler and run by tests/serve_policy_harness.cpp, which checks that every
request completes once or is rejected exactly when no slot can hold it, that placements
are aligned, inside the arenas and disjoint, that each queue is served in order, and
that bulk steps never crowd out waiting small requests."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2212_05098_amd", "csrc")


def test_policy_under_mock_executor(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no C++ compiler")
    exe = tmp_path / "harness"
    subprocess.check_call([cxx, "-std=c++17", "-O2", "-Wall", "-Wextra", "-Werror", "-I", CSRC,
                           os.path.join(HERE, "serve_policy_harness.cpp"), "-o", str(exe)])
    p = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert p.returncode == 0, p.stdout + p.stderr
    lines = p.stdout.strip().splitlines()
    assert len(lines) == 4 and all(l.startswith("ok ") for l in lines), p.stdout
