"""The host C++ of libocck (tree building, argument checks, handles) built
with g++ under AddressSanitizer and UndefinedBehaviorSanitizer and run on a
chain, a sheet and a cluster (tests/sanitize/driver.cpp).  The device-side
functions are replaced by stand-ins that report OCCK_EHIP; no HIP is
involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1708_05353_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "occk_sanitize")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-ffp-contract=off", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I" + os.path.join(ROOT, "include"),
           os.path.join(CSRC, "tree_build.cpp"), os.path.join(CSRC, "abi.cpp"),
           os.path.join(ROOT, "tests", "sanitize", "device_stubs.cpp"),
           os.path.join(ROOT, "tests", "sanitize", "driver.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and "sanitize driver OK" in r.stdout, (r.stdout[-3000:], r.stderr[-3000:])
