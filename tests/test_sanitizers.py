"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
the FP64 oracle driven through every function it exports, and the library's
host setup math (quadrature, Legendre tables, WFD / MPD Laplacians, the
factorised Fokker-Planck operator and its chunk products: what sn_setup and
the sn_diag_* calls run on the host), each built with gcc / g++ and run on
small slabs including K = 1, N = 2 and ragged chunks.  Any out-of-bounds
access, use after free, leak or undefined operation fails the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _run(cmd_build, exe, tmp_path):
    b = subprocess.run(cmd_build, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    # a sanitized executable must not inherit a preloaded library
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    out = _run(["gcc", "-std=c99", "-D_DEFAULT_SOURCE", "-fopenmp", *SAN, "-o", exe,
                os.path.join(HERE, "sanitize", "oracle_driver.c"), os.path.join(ROOT, "oracle", "sn_oracle.c"), "-lm"],
               exe, tmp_path)
    assert "oracle driver ok" in out


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_host_setup_math_under_sanitizers(tmp_path):
    exe = str(tmp_path / "setup_driver")
    csrc = os.path.join(ROOT, "paper_1907_13013_amd", "csrc")
    out = _run(["g++", "-std=c++17", *SAN, "-I", csrc, "-o", exe, os.path.join(HERE, "sanitize", "setup_driver.cpp"),
                os.path.join(csrc, "setup_math.cpp")], exe, tmp_path)
    assert "setup driver ok" in out
