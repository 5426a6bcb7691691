"""The library's host-only logic (the serving arena, option and request
checks) compiled with AddressSanitizer and UndefinedBehaviorSanitizer by the
host compiler and run on the CPU: no memory error, no undefined behaviour,
every check of tests/cpp/host_logic_check.cpp holds."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs the host C++ compiler")
def test_host_logic_under_sanitizers(tmp_path):
    exe = tmp_path / "host_logic_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_0906_3978_amd", "csrc"),
           os.path.join(ROOT, "tests", "cpp", "host_logic_check.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-3000:]
    assert run.stdout.strip().endswith("OK")
