"""The CPU code built with AddressSanitizer and UndefinedBehaviorSanitizer
(leak checking on): the oracle (tests/sanitize/oracle_check.c drives its
entry points at N = 2^8, plain and bootstrapping chains) and the library's
host-side set-up arithmetic (tests/sanitize/host_math_check.cpp: prime
chains, samplers, canonical embedding, slot-transform plans, Chebyshev
interpolants).  Any report fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-ffp-contract=off"]


def _run(cmd, tmp_path, exe):
    subprocess.check_call(cmd, cwd=tmp_path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([str(exe)], cwd=tmp_path, env=env, capture_output=True, text=True, timeout=600)
    out = p.stdout + p.stderr
    print(out)
    assert p.returncode == 0, out[-3000:]
    assert "Sanitizer" not in out and "runtime error" not in out, out[-3000:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_check"
    _run(["gcc", "-std=gnu11"] + SAN + ["-o", str(exe), os.path.join(ROOT, "tests", "sanitize", "oracle_check.c"),
                                         os.path.join(ROOT, "oracle", "ckks_oracle.c"), "-lquadmath", "-lm"],
         tmp_path, exe)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_math_under_sanitizers(tmp_path):
    exe = tmp_path / "host_math_check"
    _run(["g++", "-std=gnu++17"] + SAN + ["-o", str(exe), os.path.join(ROOT, "tests", "sanitize", "host_math_check.cpp"),
                                          os.path.join(ROOT, "paper_2606_10477_amd", "csrc", "host_math.cpp"),
                                          "-lquadmath"],
         tmp_path, exe)
