"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
the contraction and planar plan builders for every distance, the oracle's
procedures, and the sweep kernels' source on the host emulation (forward and
adjoint at d = 3, a truncated forward at d = 5), built with g++/gcc
-fsanitize=address,undefined (reports are fatal) and run in a child process."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2605_17230_amd", "csrc")
EMU = os.path.join(ROOT, "tests", "emu")
BUILD = os.path.join(ROOT, "tests", "emu", "_build")
FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


@pytest.mark.slow
def test_host_code_under_sanitizers():
    os.makedirs(BUILD, exist_ok=True)
    obj = os.path.join(BUILD, "tn_oracle_san.o")
    exe = os.path.join(BUILD, "sanitize_main")
    subprocess.check_call(["gcc", "-std=c11", *FLAGS, "-c", os.path.join(ROOT, "oracle", "tn_oracle.c"), "-o", obj])
    subprocess.check_call(["g++", "-std=c++20", *FLAGS, "-I", CSRC, "-I", EMU, os.path.join(SAN, "sanitize_main.cpp"),
                           os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "kw_plan.cpp"), obj, "-o", exe,
                           "-lpthread", "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=1200)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert "0 failures" in r.stdout
