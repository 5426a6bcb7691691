"""The C ABI used from plain C: include/wiener.h compiles as C99 and the
example program builds against the library (CPU); the program runs a solve
on the GPU and exits cleanly (GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_0906_3978_amd", "examples", "wiener_example.c")
LIBDIR = os.path.join(ROOT, "paper_0906_3978_amd")


def _build(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    if not os.path.exists(os.path.join(LIBDIR, "libwiener.so")):
        pytest.fail("libwiener.so is not built")
    exe = str(tmp_path / "wiener_example")
    cmd = [cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-O2", "-I", os.path.join(ROOT, "include"),
           SRC, "-L", LIBDIR, "-lwiener", f"-Wl,-rpath,{LIBDIR}", "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_c_example_builds(tmp_path):
    _build(tmp_path)


@pytest.mark.gpu
def test_c_example_runs(tmp_path):
    exe = _build(tmp_path)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr
    assert "iterations" in r.stdout
