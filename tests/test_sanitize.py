"""The host-side C/C++ under AddressSanitizer and UndefinedBehaviorSanitizer:
the input generator (inputs/hjgen.c), the CPU oracle (oracle/oracle.c) and
the genetic search engine (csrc/hj_ga.cpp), built with gcc/g++ into one
driver (tests/sanitize_driver.cpp) that calls every exported function,
including the error returns, with OpenMP threads on. Host code only: no GPU
code is built with a sanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1",
       "-fopenmp", "-ffp-contract=off"]


@pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None, reason="needs gcc and g++")
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    objs = []
    for src in ("paper_2002_12115_amd/inputs/hjgen.c", "oracle/oracle.c"):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.check_call(["gcc", "-std=c11", *SAN, "-c", os.path.join(ROOT, src), "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "sanitize_driver")
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "paper_2002_12115_amd", "csrc"),
                           os.path.join(ROOT, "tests", "sanitize_driver.cpp"),
                           os.path.join(ROOT, "paper_2002_12115_amd", "csrc", "hj_ga.cpp"), *objs,
                           "-o", exe, "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitize ok" in r.stdout
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr
