"""Host code of the library under the address and undefined-behaviour
sanitizers (CPU only), built with g++ from its headers: the server's pool
allocator against an independent interval model, and the server's admission
pass against its policy on random arrivals and completions."""
import os
import shutil
import subprocess

import pytest

from tests._util import ROOT

HOST = os.path.join(ROOT, "tests", "host")
CSRC = os.path.join(ROOT, "paper_2602_03857_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_pool_allocator_under_sanitizers(tmp_path):
    exe = str(tmp_path / "pool_allocator_check")
    build = subprocess.run(
        ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-I", CSRC,
         os.path.join(HOST, "pool_allocator_check.cpp"), "-o", exe],
        capture_output=True, text=True, timeout=240)
    assert build.returncode == 0, build.stderr
    run = subprocess.run([exe], capture_output=True, text=True, timeout=240,
                         env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1"})
    assert run.returncode == 0 and run.stdout.strip() == "ok", run.stdout + run.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_admission_policy_under_sanitizers(tmp_path):
    exe = str(tmp_path / "admission_check")
    build = subprocess.run(
        ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-I", CSRC,
         os.path.join(HOST, "admission_check.cpp"), "-o", exe],
        capture_output=True, text=True, timeout=240)
    assert build.returncode == 0, build.stderr
    run = subprocess.run([exe], capture_output=True, text=True, timeout=240,
                         env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1"})
    assert run.returncode == 0 and run.stdout.strip() == "ok", run.stdout + run.stderr
