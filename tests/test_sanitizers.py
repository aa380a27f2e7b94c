"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code
(libmlb's stencil tables, pair constants and linear-stability radius) and of
the float64 oracle, each run over small cases of every option it has
(tests/sanitize/*_main.*).  Any out-of-bounds access, use after free, leak
or undefined operation aborts the program with a report."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, exe, env=None):
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    e = dict(os.environ)
    e.update(env or {})
    e["ASAN_OPTIONS"] = "abort_on_error=0:halt_on_error=1"
    e["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    p = subprocess.run([exe], capture_output=True, text=True, env=e, timeout=300)
    assert p.returncode == 0, p.stdout[-2000:] + p.stderr[-4000:]
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, p.stderr[-4000:]
    return p.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not installed")
def test_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_san")
    src = [os.path.join(HERE, "sanitize", "host_main.cpp"),
           os.path.join(REPO, "paper_1105_3634_amd", "csrc", "tables.cpp"),
           os.path.join(REPO, "paper_1105_3634_amd", "csrc", "stability.cpp")]
    out = _run(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *SAN, *src, "-o", exe], exe)
    assert "host checks done" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    src = os.path.join(HERE, "sanitize", "oracle_main.c")
    out = _run(["gcc", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fopenmp", *SAN, src, "-o", exe, "-lm"],
               exe, env={"OMP_NUM_THREADS": "4"})
    assert "oracle checks done" in out and "NOT FINITE" not in out
