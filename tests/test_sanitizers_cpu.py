"""The host C/C++ code -- the oracle, the workload generator and the replay-window
cutter -- built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc / g++,
CPU only) and driven over edge inputs by tests/sanitize/driver.cpp: quantities up to
INT32_MAX, repeated and decreasing times, full sides, refused snapshots, the batch
runner on several threads, window cutting.  Any sanitizer finding fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
INC = ["-I", os.path.join(ROOT, "oracle"), "-I", os.path.join(ROOT, "paper_2308_13289_amd", "workload"),
       "-I", os.path.join(ROOT, "include")]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not shutil.which("gcc") or not shutil.which("g++"):
        pytest.skip("gcc / g++ not found")
    d = tmp_path_factory.mktemp("sanitize")
    objs = []
    for src in ("oracle/lob_oracle.c", "paper_2308_13289_amd/workload/flowgen.c"):
        o = str(d / (os.path.basename(src) + ".o"))
        subprocess.run(["gcc", "-std=c11", "-pthread", *SAN, *INC, "-c", os.path.join(ROOT, src), "-o", o],
                       check=True)
        objs.append(o)
    for src in ("paper_2308_13289_amd/csrc/lob_windows.cpp", "tests/sanitize/driver.cpp"):
        o = str(d / (os.path.basename(src) + ".o"))
        subprocess.run(["g++", "-std=c++17", "-pthread", *SAN, *INC, "-c", os.path.join(ROOT, src), "-o", o],
                       check=True)
        objs.append(o)
    exe = str(d / "driver")
    subprocess.run(["g++", "-pthread", *SAN, *objs, "-o", exe, "-lm"], check=True)
    return exe


def test_host_code_under_asan_and_ubsan(driver):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitize driver ok" in r.stdout
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr
