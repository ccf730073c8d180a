"""The bank plan (argument checks, filter-to-slot layout, per-slot FP64
coefficients, LDS geometry) is plain C++ with no HIP dependency: build it with
g++ under AddressSanitizer and UBSan and drive it with random banks, including
a template filling a whole workgroup (2,048 filters at 4 filters per lane),
templates split over several workgroups (up to 9,000 filters), templates that
fill their rows exactly, many one-filter templates and chunk lengths that are
not multiples of 16."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_layout_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "layout_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-Wall", "-Werror",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1602_05573_amd", "csrc"),
           os.path.join(ROOT, "paper_1602_05573_amd", "csrc", "layout.cpp"),
           os.path.join(ROOT, "tests", "layout_driver.cpp"), "-o", exe]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, "60"], env=env, capture_output=True, text=True, timeout=300)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "layout ok" in r.stdout
